"""pamx_swap_noalloc (the SWAP entry point that allocates nothing, its
scratch a fixed device array of the library) against pamx_swap with a
caller's workspace: the same kernels, so the same medoids, labels, TD, swap
trajectory and counts bit for bit.  Two calls in a row share the array, the
second on a smaller input; integer and FP32 matrices, FastPAM1 and eager
FastPAM2."""
import numpy as np
import pytest

from paper_2008_05171_amd import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _say(*a):
    print("[case]", *a, flush=True)


def _abi():
    from paper_2008_05171_amd import pamx
    return pamx


def _matrix(n, seed, dtype):
    import paper_2008_05171_amd as px
    if dtype == "i32":
        X = datagen.int_points(n, 2, 0, 1000, seed=seed)
    else:
        X = datagen.gaussian_mixture(n, 8, 12, seed=seed)
    return px.dist(torch.from_numpy(X).to(DEV))


def _run(fn_noalloc, D, k, start, variant, cap):
    abi = _abi()
    n = D.shape[0]
    med = torch.from_numpy(start).to(DEV)
    lab = torch.full((n,), -7, dtype=torch.int32, device=DEV)
    tbuf = torch.zeros(cap * 16, dtype=torch.uint8, device=DEV)
    opt = abi.pamx_default_options()
    opt.variant = variant
    opt.trace = tbuf.data_ptr()
    opt.trace_cap = cap
    if fn_noalloc:
        rc, td, st = abi.pamx_swap_noalloc(D, k, med, labels=lab, opt=opt)
    else:
        nb = abi.pamx_workspace_bytes(n, k, 0, abi.PAMX_INPUT_D, abi._dtype_code(D), opt)
        ws = torch.empty(nb, dtype=torch.uint8, device=DEV)
        rc, td, st = abi.pamx_swap(D, k, med, ws, labels=lab, opt=opt)
    torch.cuda.synchronize()
    return (rc, td, st.iterations, st.swaps, st.converged, med.cpu().numpy(), lab.cpu().numpy(),
            tbuf.cpu().numpy()[: 16 * st.swaps].tobytes())


@pytest.mark.parametrize("dtype", ["i32", "f32"])
@pytest.mark.parametrize("variant", [1, 2])
def test_noalloc_equals_workspace_call(dtype, variant):
    for call, (n, k, seed) in enumerate([(3000, 24, 11), (1100, 9, 12)]):
        _say("noalloc", dtype, "variant", variant, "call", call, "n", n, "k", k)
        D = _matrix(n, seed, dtype)
        start = datagen.random_subset(n, k, seed=seed + 100)
        cap = 64 * k + 64
        got = _run(True, D, k, start, variant, cap)
        want = _run(False, D, k, start, variant, cap)
        assert got[0] == want[0] == 0
        assert got[1] == want[1]                        # TD, bitwise
        assert got[2:5] == want[2:5]                    # iterations, swaps, converged
        assert np.array_equal(got[5], want[5])          # medoids
        assert np.array_equal(got[6], want[6])          # labels
        assert got[7] == want[7]                        # swap trajectory
        assert got[3] >= 1

