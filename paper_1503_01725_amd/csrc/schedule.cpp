// Host-only launch schedule of the batched runtime (see schedule.hpp).
#include "schedule.hpp"

#include <algorithm>
#include <numeric>

namespace psl {

std::vector<int32_t> assign_pipelines(const uint32_t* batch_sizes, size_t nb, int np) {
    std::vector<int32_t> pipe_of(nb, 0);
    if (np <= 1 || nb == 0) return pipe_of;
    std::vector<size_t> order(nb);
    std::iota(order.begin(), order.end(), size_t(0));
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t x, size_t y) { return batch_sizes[x] > batch_sizes[y]; });
    std::vector<uint64_t> load(size_t(np), 0);
    for (size_t i : order) {
        int best = 0;
        for (int p = 1; p < np; ++p)
            if (load[size_t(p)] < load[size_t(best)]) best = p;
        pipe_of[i] = best;
        load[size_t(best)] += batch_sizes[i];
    }
    return pipe_of;
}

std::vector<SchedOp> build_schedule(const uint32_t* batch_sizes, size_t nb, int np,
                                    uint32_t n_rep) {
    const std::vector<int32_t> pipe_of = assign_pipelines(batch_sizes, nb, np);
    std::vector<SchedOp> ops;
    ops.reserve(size_t(n_rep) * (nb + 4));
    for (uint32_t r = 0; r < n_rep; ++r) {
        if (np > 1) ops.push_back({SchedOp::kFork, -1, -1});
        for (size_t i = 0; i < nb; ++i) ops.push_back({SchedOp::kBatch, pipe_of[i], int64_t(i)});
        if (np > 1) ops.push_back({SchedOp::kJoin, -1, -1});
        ops.push_back({SchedOp::kFold, -1, -1});
        ops.push_back({SchedOp::kNextRep, -1, -1});
    }
    return ops;
}

std::string check_schedule(const std::vector<SchedOp>& ops, size_t nb, int np, uint32_t n_rep) {
    if (np < 1) return "no pipeline";
    std::vector<int> seen(nb, 0);
    bool forked = false;
    uint32_t reps = 0;
    size_t batches_in_rep = 0;
    for (size_t k = 0; k < ops.size(); ++k) {
        const SchedOp& o = ops[k];
        switch (o.kind) {
        case SchedOp::kFork:
            if (np == 1) return "fork with one pipeline";
            if (forked) return "fork while forked";
            if (batches_in_rep) return "fork after the replica's first batch";
            forked = true;
            break;
        case SchedOp::kBatch:
            if (o.batch < 0 || size_t(o.batch) >= nb) return "batch index out of range";
            if (o.pipe < 0 || o.pipe >= np) return "pipeline out of range";
            if (np > 1 && !forked) return "batch on a pipeline stream before the fork";
            if (seen[size_t(o.batch)] != int(reps)) return "batch twice in a replica";
            ++seen[size_t(o.batch)];
            ++batches_in_rep;
            break;
        case SchedOp::kJoin:
            if (!forked) return "join without fork";
            forked = false;
            break;
        case SchedOp::kFold:
            if (forked) return "fold before the join";
            if (batches_in_rep != nb) return "fold before every batch of the replica";
            break;
        case SchedOp::kNextRep:
            if (k == 0 || ops[k - 1].kind != SchedOp::kFold) return "replica not closed by a fold";
            ++reps;
            batches_in_rep = 0;
            break;
        default:
            return "unknown step";
        }
    }
    if (forked) return "schedule ends forked";
    if (reps != n_rep) return "wrong number of replicas";
    for (int c : seen)
        if (c != int(n_rep)) return "a batch missing from a replica";
    return std::string();
}

}  // namespace psl
