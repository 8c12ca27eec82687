"""psht_synth_noalloc (synthesis whose workspace is the library's static
device scratch array) against psht_synth with a caller workspace, through the
C ABI: two calls in a row on different plans, the second smaller, each within
the 10 eps parity bar of the other (they run the same kernels, so the maps
agree to the last bit), and the size limit."""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2603_17166_amd import _lib
from paper_2603_17166_amd import synthetic as syn
from paper_2603_17166_amd.plan import Plan

pytestmark = pytest.mark.gpu
DEG = math.pi / 180


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _both(plan, a, eps):
    lib = _lib.load()
    st = torch.cuda.current_stream().cuda_stream
    n = plan.npoints
    ref = torch.full((n,), complex(float("nan"), 0.0), dtype=plan.map_dtype, device="cuda")
    got = torch.full((n,), complex(float("nan"), 0.0), dtype=plan.map_dtype, device="cuda")
    ws = torch.empty(plan.info["workspace_bytes_per_map"], dtype=torch.uint8, device="cuda")
    _lib.check(lib.psht_synth(plan._h, 1, a.data_ptr(), ref.data_ptr(), ws.data_ptr(), ws.numel(), st))
    _lib.check(lib.psht_synth_noalloc(plan._h, 1, a.data_ptr(), got.data_ptr(), st))
    torch.cuda.synchronize()
    r = ref.cpu().numpy().astype(np.complex128)
    g = got.cpu().numpy().astype(np.complex128)
    assert np.all(np.isfinite(g))
    err = float(np.linalg.norm(g - r) / np.linalg.norm(r))
    say("  noalloc vs caller workspace: rel L2 %.2e, bit-identical %s" % (err, bool(np.array_equal(g, r))))
    assert err <= 10 * eps


@pytest.mark.parametrize("prec,eps", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_noalloc_matches_synth_two_calls(prec, eps):
    cases = [(256, 2, 20.0, 20000), (96, 0, 8.0, 3000)]  # the second call is smaller
    for lmax, spin, rad, n in cases:
        say("noalloc %s: lmax %d spin %d cap %g deg, %d points" % (prec, lmax, spin, rad, n))
        th, ph = syn.uniform_cap(n, rad * DEG, 9500 + lmax)
        plan = Plan(th, ph, lmax, spin, eps, prec)
        # the lmax 256 plan takes the degree-segmented synthesis (partial copies
        # of F in the scratch), the lmax 96 plan the plain work list
        say("  synthesis segment %d, partial copies %d" % (plan.info["syn_segment"], plan.info["syn_parts"]))
        assert plan.info["workspace_bytes_per_map"] <= _lib.NOALLOC_SCRATCH_BYTES
        a = torch.as_tensor(syn.gaussian_alm(lmax, spin, 9600 + lmax), device="cuda")
        _both(plan, a, eps)
        plan.close()


def test_noalloc_rejects_oversized_plan():
    th, ph = syn.uniform_cap(2000, 30 * DEG, 9700)
    plan = Plan(th, ph, 2048, 2, 1e-10, "fp64")
    assert plan.info["workspace_bytes_per_map"] > _lib.NOALLOC_SCRATCH_BYTES
    a = torch.zeros((2, syn.nalm(2048)), dtype=torch.complex128, device="cuda")
    out = torch.empty(2000, dtype=torch.complex128, device="cuda")
    code = _lib.load().psht_synth_noalloc(plan._h, 1, a.data_ptr(), out.data_ptr(),
                                           torch.cuda.current_stream().cuda_stream)
    assert code == _lib.PSHT_ERR_WORKSPACE
    assert b"static scratch" in _lib.load().psht_last_error()
    plan.close()
