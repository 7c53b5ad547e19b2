"""pic_diag_noalloc, the entry point that allocates nothing, against
pic_diag with host outputs: the same values bit for bit on two calls in a
row on one GPU (the second with fewer particles), a call with some outputs
left out, and the refusal of a context larger than its staging array."""

import numpy as np
import pytest

from paper_2102_10983_amd import workloads as W

pytestmark = pytest.mark.gpu
KEYS = ("gamma", "px", "py", "pz", "x", "k_last", "status")


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(num, seed):
    from paper_2102_10983_amd import runner
    # thermal electrons in an a0 = 60 wave: sub-cycled steps, some leave the grid
    wl = W.make_workload("noalloc", num, 60.0, 75, 400, 3, 3, 0.01, 4.0, seed=seed,
                         theta=10.0 / 511.0)
    run = runner.DeviceRun(wl, S=wl.steps, precision="fp64fast", binning="none")
    run.reset()
    run.advance(wl.steps)
    return run


def test_noalloc_equals_diag_on_two_calls(torch_gpu):
    for num, seed in ((5000, 11), (3001, 12)):
        print(f"pic_diag_noalloc vs pic_diag: {num} electrons, seed {seed}", flush=True)
        run = _run(num, seed)
        want = run.pusher.diag()
        got = run.pusher.diag_noalloc()
        part = run.pusher.diag_noalloc(keys=("px", "status"), counters=False)
        run.close()
        for k in KEYS:
            assert got[k].dtype == want[k].dtype and np.array_equal(got[k], want[k]), k
        assert got["counters"] == want["counters"]
        assert want["counters"]["lost"] > 0 and want["counters"]["n_star"] > 0
        assert set(part) == {"px", "status"}
        assert np.array_equal(part["px"], want["px"])
        assert np.array_equal(part["status"], want["status"])


def test_noalloc_refuses_more_particles_than_its_array(torch_gpu):
    from paper_2102_10983_amd import picsub
    L = picsub.load_library()
    cap = 1572864                      # PIC_DIAG_NOALLOC_MAX_NP
    p = picsub.Pusher(num=cap + 1, ncells=64, order=1, dx=0.1, dt=0.09, psi_max=0.01,
                      precision="fp64fast", binning="none")
    try:
        c = picsub.Counters()
        st = L.pic_diag_noalloc(p._ctx, None, None, None, None, None, None, None,
                                picsub.C.byref(c))
        assert st == 1, st             # PIC_E_ARG
        assert b"exceed" in L.pic_last_error(p._ctx)
    finally:
        p.close()
