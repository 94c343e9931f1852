"""The GPU direct sum (fmm_direct) against the oracle's direct sum.

Both sides compute sum_i u_i Log(y_j - x_i) on the principal branch with
coincident pairs skipped, in FP64 with compensated sums; they differ only in
how ln and Arg are rounded (the kernel's own ln/atan2 vs libm's clog) and in
the rounding of r^2.  Each term is off by a few ulp of (|ln r| + pi) |u_i|,
so the bound written here is 64 ulp of sum_i |u_i| (|ln r_max| + |ln r_min|
+ pi) per target.  Sizes span several 256-wide source tiles and target
blocks with ragged tails; every case prints its sizes first."""
import sys

import numpy as np
import pytest

from paper_1204_3105_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def F():
    from paper_1204_3105_amd import fmm
    fmm.lib()
    return fmm


def bound(xs, ys, u, xt, yt):
    d = np.hypot(np.ptp(np.concatenate([xs, xt])), np.ptp(np.concatenate([ys, yt])))
    lnmax = abs(np.log(max(d, 1e-300)))
    return 64 * 2.0 ** -52 * np.abs(u).sum() * (lnmax + 40.0 + np.pi)


def compare(orc, phi, xs, ys, u, xt, yt):
    ref = orc.direct_principal(xs, ys, u, xt, yt)
    err = np.abs(phi - ref).max() if len(ref) else 0.0
    tol = bound(xs, ys, u, xt, yt) if len(xs) else 0.0
    say("  max |gpu - oracle| %.3e (bound %.3e)" % (err, tol))
    assert err <= tol
    return ref


@pytest.mark.parametrize("n,seed", [(1, 1), (255, 2), (3001, 3), (5120, 4)])
def test_direct_same_points_host(F, orc, n, seed):
    w = inputs.uniform_square(n, seed=seed)
    say("direct same points N=%d seed=%d (host pointers)" % (n, seed))
    phi = F.direct(w.xs, w.ys, w.u)
    compare(orc, phi, w.xs, w.ys, w.u, w.xs, w.ys)


def test_direct_separate_clustered_host(F, orc):
    w = inputs.gaussian_mixture(4097, 1031, seed=5)
    # some targets sit exactly on sources, some on the branch cut of a source
    xt, yt = w.xt.copy(), w.yt.copy()
    xt[:7], yt[:7] = w.xs[:7], w.ys[:7]
    xt[7:11], yt[7:11] = w.xs[20:24] - 0.25, w.ys[20:24]
    say("direct gaussian mixture N=4097 -> M=1031 (host pointers)")
    phi = F.direct(w.xs, w.ys, w.u, xt, yt)
    ref = compare(orc, phi, w.xs, w.ys, w.u, xt, yt)
    assert np.all(np.isfinite(phi)) and np.all(np.isfinite(ref))


def test_direct_device_on_torch_stream(F, orc):
    import torch
    w = inputs.uniform_square(20011, seed=6, m=6007, targets_same=False)
    say("direct N=20011 -> M=6007 (device pointers, torch stream)")
    dev = torch.device("cuda:0")
    src = torch.tensor(w.xs + 1j * w.ys, dtype=torch.complex128, device=dev)
    tgt = torch.tensor(w.xt + 1j * w.yt, dtype=torch.complex128, device=dev)
    u = torch.tensor(w.u, dtype=torch.float64, device=dev)
    phi = F.direct(None, None, u, src=src, tgt=tgt).cpu().numpy()
    compare(orc, phi, w.xs, w.ys, w.u, w.xt, w.yt)
    # same tensor as targets: coincident pairs skipped
    phi2 = F.direct(None, None, u, src=src, tgt=src).cpu().numpy()
    idx = inputs.subsample(len(w.xs), 512, 9)
    ref2 = orc.direct_principal(w.xs, w.ys, w.u, w.xs[idx], w.ys[idx])
    err = np.abs(phi2[idx] - ref2).max()
    say("  same-tensor targets, 512 sampled: max err %.3e" % err)
    assert err <= bound(w.xs, w.ys, w.u, w.xs, w.ys)


def test_direct_edge_cases(F, orc):
    say("direct edge cases: no sources, no targets, branch cut, one point")
    z = F.direct(np.zeros(0), np.zeros(0), np.zeros(0), np.array([0.5, 0.1]), np.array([0.5, 0.2]))
    assert z.shape == (2,) and np.all(z == 0)
    e = F.direct(np.array([0.5]), np.array([0.5]), np.array([2.0]), np.zeros(0), np.zeros(0))
    assert e.shape == (0,)
    # target left of the source on the same horizontal line: Arg = pi exactly
    b = F.direct(np.array([0.5]), np.array([0.25]), np.array([1.0]), np.array([0.25]), np.array([0.25]))
    assert b[0].imag == np.pi and abs(b[0].real - np.log(0.25)) <= 4e-16
    one = F.direct(np.array([0.3]), np.array([0.3]), np.array([1.0]))
    assert one[0] == 0
