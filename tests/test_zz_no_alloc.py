"""The allocation-free MTTKRP entry point (mttkrp_noalloc) against the
allocating one (mttkrp): the same kernels, so the results must be equal bit
for bit; two calls in a row on one GPU, the second on a smaller input (the
shared carry scratch keeps the first call's contents); a mode whose carry
scratch exceeds the fixed array is refused before anything runs."""
import numpy as np
import pytest
import torch

from paper_1910_02371_amd import workloads as W
from gpu_helpers import dev_factor, dev_idx, dev_vals

pytestmark = pytest.mark.gpu


def _check_equal(tt, ix, A, s, s_order, n, R, fdt_t, accumulate=False):
    I = ix.dims[n]
    ref = torch.full((I, R), 0.25, dtype=fdt_t, device="cuda")
    out = torch.full((I, R), 0.25, dtype=fdt_t, device="cuda")
    tt.mttkrp(ix, s, A, n, out=ref, s_order=s_order, accumulate=accumulate)
    tt.mttkrp_noalloc(ix, s, A, n, out, s_order=s_order, accumulate=accumulate)
    torch.cuda.synchronize()
    assert torch.equal(out, ref), f"mode {n}: noalloc differs from mttkrp"


@pytest.mark.parametrize("form", ["f32", "bf16", "f64"])
def test_noalloc_mttkrp_matches_mttkrp_two_calls(gpu_lib, form):
    tt = gpu_lib
    dense = torch.float64 if form == "f64" else torch.float32
    # first call: heavy rows (thousands of nonzeros: many carry slots) at R 64
    big = W.random_tensor((4, 300, 200), 30000, 3, rank=3)
    ixb = tt.build_index(dev_idx(big.idx), big.dims, dev_vals(big.t, form))
    Ab = [dev_factor(a, form) for a in W.init_factors(big.dims, 64, 1.0, 5, dtype=np.float64)]
    # second call: a smaller tensor with fewer and shorter heavy rows at R 13
    # (element path), reading a scratch that still holds the first call's data
    small = W.random_tensor((3, 40, 30), 3000, 4, rank=3)
    ixs = tt.build_index(dev_idx(small.idx), small.dims, dev_vals(small.t, form))
    As = [dev_factor(a, form) for a in W.init_factors(small.dims, 13, 1.0, 6, dtype=np.float64)]
    for n in range(3):
        _check_equal(tt, ixb, Ab, tt.INDEX_T, tt.ORDER_COO, n, 64, dense)
        _check_equal(tt, ixs, As, tt.INDEX_T, tt.ORDER_COO, n, 13, dense)
    # COO-order weights and accumulation
    w = dev_vals(np.random.default_rng(1).standard_normal(small.nnz), form)
    for n in range(3):
        _check_equal(tt, ixs, As, w, tt.ORDER_COO, n, 13, dense, accumulate=True)
    ixb.close()
    ixs.close()


def test_noalloc_mttkrp_refuses_oversized_scratch(gpu_lib):
    """A fully observed 8 x 2048 x 2048 tensor (33.5M nonzeros, 4M per
    mode-0 row) cut into 512-nonzero pieces: at R = 64 its 65,536 pieces
    need more than the 32 MiB array and the call is refused with the output
    untouched; at R = 32 they fit and the result equals mttkrp's."""
    tt = gpu_lib
    dims = (8, 2048, 2048)
    m = dims[0] * dims[1] * dims[2]
    key = W.rng_for(11).permutation(m).astype(np.int64)
    idx = [(key // (dims[1] * dims[2])).astype(np.int32),
           ((key // dims[2]) % dims[1]).astype(np.int32), (key % dims[2]).astype(np.int32)]
    t = np.random.default_rng(2).random(m).astype(np.float32)
    ix = tt.build_index(dev_idx(idx), dims, dev_vals(t, "f32"))
    ix.tune(chunk=512)
    A64 = [torch.rand(d, 64, device="cuda") for d in dims]
    out = torch.full((dims[0], 64), 7.0, device="cuda")
    with pytest.raises(tt.TTError) as e:
        tt.mttkrp_noalloc(ix, tt.INDEX_T, A64, 0, out)
    assert e.value.status == -6 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all()), "a refused call wrote its output"
    A32 = [a[:, :32].contiguous() for a in A64]
    for n in range(3):
        _check_equal(tt, ix, A32, tt.INDEX_T, tt.ORDER_COO, n, 32, torch.float32)
    ix.close()
