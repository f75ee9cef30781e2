"""The allocation-free inner product (tt_contract_inner_noalloc) against the
allocating entry point (tt_contract_inner) through the C ABI: the same
kernels on the same inputs give the same result bit for bit, on two calls in
a row whose second input is smaller (the fixed scratch keeps the first
call's contents), in FP64, FP32 and BF16; both within tolerance of the FP64
oracle; oversize pairs refused before any launch; no device memory taken."""
import pytest

from oracle import tt_oracle as O

from helpers import TOL, random_pair, scalar_err, to_gpu, tt_norm

pytestmark = pytest.mark.gpu

# (modes, ranks of X, ranks of Y): an order-10 rank-32 pair, then a smaller
# order-5 pair; both take the paths that use a workspace (two half sweeps)
BIG = ([16] * 10, [1] + [32] * 9 + [1], [1] + [32] * 9 + [1])
SMALL = ([3, 5, 2, 7, 4], [1, 3, 17, 5, 2, 1], [1, 9, 2, 33, 6, 1])


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_noalloc_matches_allocating_entry(ttc, dtype):
    import torch
    cases = []
    for n, (modes, rx, ry) in enumerate((BIG, SMALL)):
        x, y = random_pair(808 + n, modes, rx, ry)
        xg, xs = to_gpu(x, dtype)
        yg, ys = to_gpu(y, dtype)
        want = float(ttc.tt_contract_inner(xg, yg).item())
        cases.append((xg, yg, xs, ys, want))
    outs = [torch.full((), float("nan"), dtype=torch.float64, device="cuda") for _ in cases]
    torch.cuda.synchronize()
    for (xg, yg, _, _, _), out in zip(cases, outs):
        ttc.tt_contract_inner_noalloc(xg, yg, out)
    torch.cuda.synchronize()
    for (xg, yg, xs, ys, want), out in zip(cases, outs):
        got = float(out.item())
        assert got == want
        tol = TOL["f32"] if dtype == "bf16" else TOL[dtype]
        assert scalar_err(got, O.inner_lr(xs, ys), tt_norm(xs), tt_norm(ys)) <= tol


def test_noalloc_takes_no_device_memory(ttc):
    import torch
    x, y = random_pair(811, *BIG)
    xg, _ = to_gpu(x, "f32")
    yg, _ = to_gpu(y, "f32")
    out = torch.empty((), dtype=torch.float64, device="cuda")
    ttc.tt_contract_inner_noalloc(xg, yg, out)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(5):
        ttc.tt_contract_inner_noalloc(xg, yg, out)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0


def test_noalloc_refuses_oversize_workspace(ttc):
    import torch
    modes, r = [64] * 12, [1] + [128] * 11 + [1]
    # workspace of the two half sweeps: the reversed prefix alone is
    # 6 cores x 128 x 64 x 128 FP32 = 25 MB, beyond the 16 MiB scratch
    xg = [torch.zeros(r[k], modes[k], r[k + 1], dtype=torch.float32, device="cuda") for k in range(12)]
    out = torch.full((), -1.0, dtype=torch.float64, device="cuda")
    with pytest.raises(ttc.TTCError) as ei:
        ttc.tt_contract_inner_noalloc(xg, xg, out)
    assert ei.value.name == "TTC_ERR_WORKSPACE"
    assert out.item() == -1.0
