"""The clinical-shape workloads: the paper's H&N and prostate voxel sizes,
the plan shapes (a couch-90 field among five coplanar ones; seven coplanar
fields), every material present, the phantoms centred on the isocentre."""
import numpy as np

from paper_1503_01725_amd import workloads as wl


def test_head_and_neck_workload():
    W = wl.workload("hn_6beam")
    ph = W.phantom
    assert ph.vox == (0.137, 0.125, 0.137)
    nz, ny, nx = ph.density.shape
    ext = np.array([nx, ny, nz]) * np.array(ph.vox)
    assert np.allclose(np.array(ph.origin), -ext / 2)
    assert set(np.unique(ph.density).astype(np.float64).round(4).tolist()) == {0.0012, 1.04, 1.6, 1.85}
    couch = [b.couch_deg for b in W.beams]
    assert couch.count(90.0) == 1 and couch.count(0.0) == 5
    assert all(4.0 <= b.x2 - b.x1 <= 8.0 for b in W.beams)


def test_prostate_workload():
    W = wl.workload("prostate_7beam")
    ph = W.phantom
    assert ph.vox == (0.195, 0.25, 0.195)
    assert set(np.unique(ph.density).astype(np.float64).round(4).tolist()) == {0.0012, 1.02, 1.85}
    g = [b.gantry_deg for b in W.beams]
    assert len(g) == 7 and np.allclose(np.diff(g), 360.0 / 7)
    assert all(b.couch_deg == 0.0 for b in W.beams)


def test_table1_water_workload():
    """Table 1's water phantom: 240 x 240 x 300 voxels of 0.25 x 0.25 x 0.2 cm,
    top face at z = 0 centred on the isocentre."""
    W = wl.workload("water240_table1")
    ph = W.phantom
    assert ph.vox == (0.25, 0.25, 0.2)
    assert ph.density.shape == (300, 240, 240)
    assert np.allclose(ph.origin, (-30.0, -30.0, 0.0))
    assert float(ph.density.min()) == float(ph.density.max()) == 1.0
    assert len(W.beams) == 1 and W.beams[0].x2 - W.beams[0].x1 == 10.0
