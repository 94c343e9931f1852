"""fmm_direct_noalloc (the direct sum with the library's fixed scratch) against
fmm_direct, its allocating counterpart, through the C ABI.

Both run the same kernels with the same slicing of the sources, so the
outputs must be bitwise equal; they are also checked against the oracle's
direct sum with the bound of the direct-sum tests (64 ulp of
sum |u| (|ln r_max| + 40 + pi) per target).  Two calls in a row, the second
smaller, share the one scratch array; a third call reuses it after an
allocating call in between.  Sizes give many source slices (so the scratch
is used) with ragged tails."""
import sys

import numpy as np
import pytest

from paper_1204_3105_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bound(xs, ys, u, xt, yt):
    d = np.hypot(np.ptp(np.concatenate([xs, xt])), np.ptp(np.concatenate([ys, yt])))
    lnmax = abs(np.log(max(d, 1e-300)))
    return 64 * 2.0 ** -52 * np.abs(u).sum() * (lnmax + 40.0 + np.pi)


def test_noalloc_equals_direct_twice_then_smaller(orc):
    import torch
    from paper_1204_3105_amd import fmm as F
    F.lib()
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream()
    cases = [(5120, 3001, 11), (2000, 700, 12), (257, 130, 13)]
    outs = []
    for ns, nt, seed in cases:
        say("noalloc case n_src=%d n_tgt=%d seed=%d" % (ns, nt, seed))
        w = inputs.uniform_square(ns, seed=seed, m=nt, targets_same=False)
        src = torch.tensor(w.xs + 1j * w.ys, dtype=torch.complex128, device=dev)
        tgt = torch.tensor(w.xt + 1j * w.yt, dtype=torch.complex128, device=dev)
        u = torch.tensor(w.u, dtype=torch.float64, device=dev)
        out = torch.full((nt,), complex(np.nan, np.nan), dtype=torch.complex128, device=dev)
        F.direct_noalloc(src, tgt, u, out, stream=st)
        outs.append((w, out))
    torch.cuda.synchronize()
    for (ns, nt, seed), (w, out) in zip(cases, outs):
        src = torch.tensor(w.xs + 1j * w.ys, dtype=torch.complex128, device=dev)
        tgt = torch.tensor(w.xt + 1j * w.yt, dtype=torch.complex128, device=dev)
        u = torch.tensor(w.u, dtype=torch.float64, device=dev)
        ref_gpu = F.direct(None, None, u, src=src, tgt=tgt)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        want = ref_gpu.cpu().numpy()
        assert np.array_equal(got.view(np.float64), want.view(np.float64)), (ns, nt)
        ref = orc.direct_principal(w.xs, w.ys, w.u, w.xt, w.yt)
        err = float(np.abs(got - ref).max())
        say("noalloc n_src=%d n_tgt=%d max abs vs oracle %.3e (bound %.3e)" %
            (ns, nt, err, bound(w.xs, w.ys, w.u, w.xt, w.yt)))
        assert err <= bound(w.xs, w.ys, w.u, w.xt, w.yt)
    # after allocating calls, the scratch is still this device's and reusable
    w, out = outs[1]
    src = torch.tensor(w.xs + 1j * w.ys, dtype=torch.complex128, device=dev)
    tgt = torch.tensor(w.xt + 1j * w.yt, dtype=torch.complex128, device=dev)
    u = torch.tensor(w.u, dtype=torch.float64, device=dev)
    again = torch.empty_like(out)
    F.direct_noalloc(src, tgt, u, again, stream=st)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(again), torch.view_as_real(out))


def test_noalloc_edges():
    import ctypes as C
    import torch
    from paper_1204_3105_amd import fmm as F
    L = F.lib()
    dev = torch.device("cuda:0")
    say("noalloc edges: no targets, no sources, bad sizes")
    # no targets: a no-op
    assert L.fmm_direct_noalloc(None, 0, None, 0, None, None, None) == 0
    assert L.fmm_direct_noalloc(None, -1, None, 0, None, None, None) == 1
    # no sources: Phi = 0
    tgt = torch.tensor([0.25 + 0.5j, 0.75 + 0.125j], dtype=torch.complex128, device=dev)
    out = torch.full((2,), complex(7.0, 7.0), dtype=torch.complex128, device=dev)
    st = torch.cuda.current_stream()
    assert L.fmm_direct_noalloc(None, 0, C.c_void_p(tgt.data_ptr()), 2, None, C.c_void_p(out.data_ptr()),
                                C.c_void_p(st.cuda_stream)) == 0
    torch.cuda.synchronize()
    assert torch.count_nonzero(torch.view_as_real(out)).item() == 0
