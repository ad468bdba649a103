"""xm_spmm_noalloc (the product entry point that allocates nothing) against
xm_spmm, through the C ABI: same kernels, so the results must be bitwise equal,
on two calls in a row (the second smaller, on the same fixed scratch), for
every stored precision and product kernel, and at the benchmark's size."""
import numpy as np
import pytest

import scenes

from conftest import progress

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _xm():
    import paper_2502_04640_amd as xm
    xm.load_library()
    return xm


def _say(msg):
    print(msg, flush=True)
    progress(msg)


def _build(sc, keep):
    xm = _xm()
    return xm.build_Q(sc.N, sc.M, torch.from_numpy(sc.frame).cuda(), torch.from_numpy(sc.landmark).cuda(),
                      torch.from_numpy(sc.u).cuda(), torch.from_numpy(sc.w).cuda(), keep=keep)


def _pair(P, dtype, r, seed):
    rng = np.random.default_rng(seed)
    Y = torch.from_numpy(rng.standard_normal((r, P.n3))).cuda()
    ref = P.spmm(Y, dtype)
    out = torch.full_like(Y, float("nan"))
    P.spmm_noalloc(Y, out, dtype)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("kind", ["upper", "full", "factored"])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_noalloc_matches_spmm_two_calls(kind, dtype):
    if kind == "factored" and dtype == "bf16":
        pytest.skip("no BF16 factored product")
    _say(f"case: noalloc {dtype} {kind}: 700 frames r=5, then 60 frames r=2")
    big = _build(scenes.random_scene(700, 12000, L=4, sigma=0.02, seed=17), ("f32", "bf16"))
    small = _build(scenes.random_scene(60, 1500, L=4, sigma=0.02, seed=18), ("f32", "bf16"))
    for P, r, seed in ((big, 5, 1), (small, 2, 2)):
        P.set_spmm_kind(dtype, kind)
        ref, out = _pair(P, dtype, r, seed)
        assert np.isfinite(out).all()
        assert np.array_equal(out, ref), float(np.abs(out - ref).max())


def test_noalloc_benchmark_size_and_limit():
    _say("case: noalloc at N=10155 (FP32 r=5 dense, FP32 factored, FP64 r=8 over the limit)")
    xm = _xm()
    P = _build(scenes.make_scene("large", 0), ("f32",))
    need = P.spmm_noalloc_bytes(5, "f32")
    assert need <= xm.api.XM_NOALLOC_SCRATCH_BYTES
    ref, out = _pair(P, "f32", 5, 3)
    assert np.array_equal(out, ref)
    P.set_spmm_kind("f32", "factored")
    ref, out = _pair(P, "f32", 5, 4)
    assert np.array_equal(out, ref)
    # the FP64 dense product at r = 8 needs more than the array: rejected before any work
    assert P.spmm_noalloc_bytes(8, "f64") > xm.api.XM_NOALLOC_SCRATCH_BYTES
    Y = torch.zeros((8, P.n3), dtype=torch.float64, device="cuda")
    out = torch.full_like(Y, 7.0)
    with pytest.raises(xm.XMError, match="XM_EINVAL"):
        P.spmm_noalloc(Y, out, "f64")
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
