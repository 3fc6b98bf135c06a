"""td_util_gemm_noalloc (no allocation; scratch in a fixed device array)
against td_util_gemm, through the C ABI: two calls in a row on one stream,
the second smaller (the array keeps the first call's contents, which must
not leak into the second), in FP64 and split-bf16. The two entry points run
the same kernels on the same padded operands, so the results agree bit for
bit."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_noalloc_gemm_matches_td_util_gemm(precision):
    import torch
    from paper_1912_03174_amd import tddftb as T
    prec = T.TD_FP64 if precision == "fp64" else T.TD_SPLIT_BF16
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    for (m, n, k), pad in (((700, 520, 900), 3), ((130, 47, 300), 0)):
        say(f"noalloc gemm {precision} {m}x{n}x{k} (leading-dimension padding {pad})")
        A = W.random_matrix(m, k, seed=m + 3 * k)
        B = W.random_matrix(k, n, seed=n + 5 * k)
        ref = T.td_util_gemm(A, B, precision=prec, n_slices=4)
        lda, ldb, ldc = k + pad, n + pad, n + 2 * pad
        Ad = torch.zeros((m, lda), dtype=torch.float64, device=dev)
        Bd = torch.zeros((k, ldb), dtype=torch.float64, device=dev)
        Ad[:, :k] = torch.from_numpy(A)
        Bd[:, :n] = torch.from_numpy(B)
        Cd = torch.full((m, ldc), 7.0, dtype=torch.float64, device=dev)   # padding must survive
        torch.cuda.synchronize()
        T.td_util_gemm_noalloc(m, n, k, Ad.data_ptr(), lda, Bd.data_ptr(), ldb, Cd.data_ptr(),
                               ldc, precision=prec, n_slices=4, stream=stream.cuda_stream)
        stream.synchronize()
        C = Cd.cpu().numpy()
        assert np.array_equal(C[:, :n], ref)
        assert np.all(C[:, n:] == 7.0)
        # the product itself: within the precision's bound of the exact product
        exact = A @ B
        scale = np.abs(A).max() * np.abs(B).max() * k
        assert np.abs(C[:, :n] - exact).max() < (1e-14 if precision == "fp64" else 1e-9) * scale
