"""tffr_entropy_step_noalloc (the step in the library's static scratch array) against
tffr_entropy_step (the step in a caller workspace), through the C ABI: the same kernels on
the same inputs, so the outputs are bit-identical.  Two calls in a row, the second on a
smaller problem (the array keeps the first call's contents), and a problem too large for
the array is refused without running."""

import numpy as np
import pytest
import torch

from paper_1910_10908_amd import _lib
from paper_1910_10908_amd import scenes
from paper_1910_10908_amd import tffr as T
from tests.gpu_helpers import DEV, Case

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu(gpu):
    print(flush=True)
    yield


def _inputs(case, n):
    s, st = case.samples()
    ph = case.real(case.rng.normal(0, 0.5, n))
    da = case.real(case.rng.normal(0, 0.004, n))
    return st, ph, da


def test_noalloc_step_matches_workspace_step():
    big = Case(512, 1024, 1024, fov=400.0, seed=301)  # the benchmark's workload
    small = Case(20, 90, 64, seed=302)
    ib, is_ = _inputs(big, 512), _inputs(small, 20)
    print("no-alloc step: 512 x 1024 -> 1024^2, then 20 x 90 -> 64^2", flush=True)
    got_big = [x.clone() for x in big.plan.tffr_entropy_step_noalloc(*ib)]
    got_small = [x.clone() for x in small.plan.tffr_entropy_step_noalloc(*is_)]
    torch.cuda.synchronize()
    for case, inp, got in ((big, ib, got_big), (small, is_, got_small)):
        ref = case.plan.tffr_entropy_step(*inp)
        for name, a, b in zip(("image", "loss", "grad_samples", "grad_phase", "grad_dalong"), got, ref):
            assert torch.equal(a, b), f"{case.prm.n_pulses} x {case.prm.n_freq}: {name}"
    # and once more on the large problem after the small one (no stale state is read)
    again = big.plan.tffr_entropy_step_noalloc(*ib)
    for a, b in zip(again, got_big):
        assert torch.equal(a, b)


def test_noalloc_step_refuses_problems_beyond_the_array():
    wl = scenes.WORKLOADS["precision_2k"]  # range spectra alone: 2048 x 2048 x 8 B = 32 MiB
    k, ku = scenes.radar_sampling(wl.n_pulses, wl.n_freq)
    prm = T.default_params(n_pulses=wl.n_pulses, n_freq=wl.n_freq, mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov)
    plan = T.Plan(prm, k, ku, DEV)
    st = torch.zeros((wl.n_pulses, wl.n_freq), dtype=torch.complex64, device=DEV)
    img = torch.empty(plan.shape_image, dtype=torch.complex64, device=DEV)
    loss = torch.empty((), dtype=torch.float64, device=DEV)
    gs = torch.empty_like(st)
    rc = plan.lib.tffr_entropy_step_noalloc(plan.handle, T._ptr(st), None, None, None, T._ptr(img), T._ptr(loss),
                                            T._ptr(gs), None, None, T._stream())
    assert rc == _lib.TFFR_ERR_SCRATCH
