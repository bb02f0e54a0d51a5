// Launch schedule of the batched runtime, as plain host data: which
// pipeline (stream) each batch of a replica runs on, and the order of the
// fork, launch, join and fold steps.  Built and checked here without any HIP
// call, so that the bookkeeping can be exercised on the CPU (under address
// and undefined-behaviour sanitizers); the runtime only executes it.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace psl {

struct SchedOp {
    enum Kind : uint8_t {
        kFork,       // record the fork event on the main stream; pipelines 0..np-1 wait on it
        kBatch,      // sample + transport batch `batch` on pipeline `pipe`
        kJoin,       // pipelines record their join events; the main stream waits on each
        kFold,       // fold the replica's energies on the main stream
        kNextRep     // advance the device replica counter on the main stream
    };
    Kind kind;
    int32_t pipe;    // kBatch: pipeline; otherwise -1
    int64_t batch;   // kBatch: batch index; otherwise -1
};

// Batches to pipelines, largest first onto the least loaded one (cost ~
// histories; ties to the lower pipeline).  np >= 1; with np == 1 every batch
// runs on pipeline 0.
std::vector<int32_t> assign_pipelines(const uint32_t* batch_sizes, size_t nb, int np);

// The steps of n_rep replicas of nb batches over np pipelines: per replica a
// fork (np > 1), the batches in plan order on their pipelines, a join
// (np > 1), the fold and the replica increment.
std::vector<SchedOp> build_schedule(const uint32_t* batch_sizes, size_t nb, int np,
                                    uint32_t n_rep);

// Empty if `ops` is a well-formed schedule of n_rep replicas of nb batches
// over np pipelines (every batch once per replica on a pipeline in [0, np),
// forks and joins balanced, a fold closing every replica after its join);
// otherwise what is wrong.
std::string check_schedule(const std::vector<SchedOp>& ops, size_t nb, int np, uint32_t n_rep);

}  // namespace psl
