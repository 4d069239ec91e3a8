"""The no-allocation apply (mudiff_matvec_noalloc, static device scratch)
against mudiff_matvec through the C ABI: same results on two calls in a row,
the second with a smaller input, on the one-lane path (uniform N_p <= 12) and
the generic path (uneven N_p), for A, L and L^T; and its host-side refusals
(R >= 8 on the matrix cores, scratch beyond its size)."""
import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _noalloc(pr, x, R, op):
    from paper_1409_8186_amd import _lib
    lib = _lib.load()
    y = pr.empty(R)
    st = lib.mudiff_matvec_noalloc(pr.h, R, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                   op, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _lib.check(st)
    return y


def test_noalloc_apply_matches_matvec():
    from paper_1409_8186_amd import Problem
    assert torch.cuda.is_available()
    lane = synth.small_random(41, 30, 0.5, 0.5, 30.0, 0.2, 6.0, 5)     # uniform N_p: one lane per pair
    lane.n_modes[:] = 9
    gen = synth.small_random(42, 17, 0.3, 1.0, 14.0, 0.1, 7.0, 4)      # uneven N_p: generic kernel
    for cl in (lane, gen):
        pr = Problem.from_cluster(cl)
        rng = np.random.default_rng(cl.M)
        for op in (1, 0, 2):
            for R in (5, 2):              # two calls in a row, the second smaller
                X = rng.normal(size=(R, cl.n_tot)) + 1j * rng.normal(size=(R, cl.n_tot))
                x = torch.tensor(X.ravel(), device="cuda")
                y0 = _noalloc(pr, x, R, op)
                y1 = pr.matvec(x, R=R, op=op)
                torch.cuda.synchronize()
                a, b = y0.cpu().numpy(), y1.cpu().numpy()
                err = np.linalg.norm(a - b) / np.linalg.norm(b)
                print(cl.M, op, R, err, flush=True)
                assert err < 1e-12, (cl.M, op, R, err)


def test_noalloc_refusals():
    from paper_1409_8186_amd import Problem, _lib
    lib = _lib.load()
    cl = synth.small_random(43, 6, 0.3, 1.0, 8.0, 0.1, 5.0, 4)
    pr = Problem.from_cluster(cl)
    x = pr.empty(8)
    y = pr.empty(8)
    st = lib.mudiff_matvec_noalloc(pr.h, 8, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                   1, None)
    assert st == 1 and b"mudiff_matvec" in lib.mudiff_last_error()
    big = synth.multi_rhs()           # 1000 disks, R = 7: generic partial sums of about 71 MiB
    pb = Problem.from_cluster(big)
    xb = pb.empty(7)
    yb = pb.empty(7)
    st = lib.mudiff_matvec_noalloc(pb.h, 7, ctypes.c_void_p(xb.data_ptr()), ctypes.c_void_p(yb.data_ptr()),
                                   1, None)
    assert st == 3 and b"scratch" in lib.mudiff_last_error()
