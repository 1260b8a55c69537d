"""fc_scan_no_alloc: the scan for callers that cannot allocate, its scratch in
the library's static per-device array.  Its results must equal fc_scan's bit
for bit, call after call (the array keeps the previous call's contents), in
every form, with and without the optional outputs; a K whose scratch would
not fit the array is refused before any device work."""
from __future__ import annotations

import numpy as np
import pytest

import fcgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FORMS = {"fp64": 1, "fp32": 2, "split_bf16": 4, "split_fp16": 8}


@pytest.fixture(scope="module")
def fc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2002_07858_amd as fc
    fc.lib()
    return fc


@pytest.fixture(scope="module")
def setup(fc):
    pr = fcgen.make_problem("c2", K=1500, true_subset=[0, 100])
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=1 | 2 | 4 | 8)
    yield pr, g
    g.destroy()


def outputs(K, drop=()):
    o = {k: torch.full((K,), -3.0, dtype=torch.float64, device="cuda")
         for k in ("dchi2", "chi2_min", "chi2_p")}
    o["argmin"] = torch.full((K,), -3, dtype=torch.int64, device="cuda")
    args = {k: (None if k in drop else v) for k, v in o.items()}
    return o, args


def run(fc, entry, g, form, d_t, p_t, drop=()):
    o, a = outputs(d_t.shape[0], drop)
    entry(g, form, d_t, p_t, a["dchi2"], a["chi2_min"], a["argmin"], a["chi2_p"])
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("drop", [(), ("chi2_min", "chi2_p"), ("chi2_min", "argmin", "chi2_p")])
def test_no_alloc_equals_fc_scan_on_two_calls(fc, setup, form, drop):
    pr, g = setup
    d_all = torch.as_tensor(pr.d).cuda()
    p_all = torch.as_tensor(pr.p_idx).cuda()
    # two calls in a row, the second with fewer universes (a different slice)
    for lo, hi in ((0, 3000), (1100, 1877)):
        d_t, p_t = d_all[lo:hi].contiguous(), p_all[lo:hi].contiguous()
        ref = run(fc, fc.fc_scan, g, FORMS[form], d_t, p_t)
        got = run(fc, fc.fc_scan_no_alloc, g, FORMS[form], d_t, p_t, drop)
        for k in ref:
            if k in drop:
                assert np.all(got[k] == -3), (form, drop, k)
            else:
                np.testing.assert_array_equal(got[k], ref[k], err_msg=f"{form} {drop} {k}")


def test_no_alloc_fp64_fewer_chunks_same_result(fc):
    """The FP64 form's chunk minima must fit the static array: on the 60^3
    grid with 40 000 universes fc_scan takes 106 chunks of at most 2048 points
    (68 MB of minima), the no-allocation entry only as many as fit 32 MiB; the
    minima merge in grid order with the strict "<", so both give the same
    results bit for bit."""
    pr = fcgen.make_problem("c3", K=20000, true_subset=[0, 1])
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=1)
    d_t = torch.as_tensor(pr.d).cuda()
    p_t = torch.as_tensor(pr.p_idx).cuda()
    assert d_t.shape[0] * (pr.G // 2048) * 16 > fc.FC_NO_ALLOC_SCRATCH_BYTES
    ref = run(fc, fc.fc_scan, g, 1, d_t, p_t)
    got = run(fc, fc.fc_scan_no_alloc, g, 1, d_t, p_t)
    for k in ref:
        np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
    assert np.all(np.isfinite(ref["dchi2"]))
    g.destroy()


def test_no_alloc_refuses_a_k_beyond_its_scratch(fc):
    """NULL chi2_min and chi2_p need 16 bytes per universe: 2^21 + 1 universes
    exceed the 32 MiB array, and the call fails before any device work."""
    pr = fcgen.make_problem("c1", K=1, true_subset=[0])
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=2)
    K = fc.FC_NO_ALLOC_SCRATCH_BYTES // 16 + 1
    d = torch.zeros((K, pr.N), dtype=torch.float64, device="cuda")
    p = torch.zeros(K, dtype=torch.int64, device="cuda")
    out = torch.full((K,), -3.0, dtype=torch.float64, device="cuda")
    with pytest.raises(fc.FCError) as ei:
        fc.fc_scan_no_alloc(g, 2, d, p, out)
    assert ei.value.code == fc.FC_ERR_INVALID_ARG
    assert "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((out == -3.0).all())          # nothing was enqueued
    # with chi2_min and chi2_p given, the FP32 form needs no scratch at all
    cm = torch.empty(K, dtype=torch.float64, device="cuda")
    cp = torch.empty(K, dtype=torch.float64, device="cuda")
    fc.fc_scan_no_alloc(g, 2, d[:4096].contiguous(), p[:4096].contiguous(), out[:4096], cm[:4096],
                        None, cp[:4096])
    torch.cuda.synchronize()
    g.destroy()
