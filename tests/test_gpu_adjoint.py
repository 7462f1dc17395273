"""GPU reverse mode (dfc_lrr_backward) against the oracle's hand-written reverse
sweep (literal Z-step form, SVD-based thresholding derivative) and against
central finite differences of the GPU forward map.

Loss L = ||W o |Z| ||_F^2 with a seeded W ~ U[0, 1]^{n x n}, so dL/dZ = 2 W^2 o Z.
Tolerances: FP64 forward vs the oracle gradient, relative Frobenius error of dM
and relative error of dlambda <= 1e-7 (both sides FP64; the eigen-decomposition
of the Gram matrix and the SVD agree to rounding); finite differences with
h = 1e-6 agree to 1e-5 relative (truncation h^2 and rounding 1e-16/h)."""
import numpy as np
import pytest

from gpu_util import need_gpu, one_thread, rel, say

pytestmark = pytest.mark.gpu


def _opts(B, iters, every, prec=0, **kw):
    return B.lrr_opts_default(precision=prec, fixed_iters=iters, checkpoint_every=every,
                              save_for_backward=1, **kw)


def _gpu_grad(B, torch, p, W, opts):
    Mt = B.to_device_colmajor(p.M)
    Zt, _, info = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, opts=opts, want_S=False)
    Wt = torch.from_numpy(np.ascontiguousarray(W.T)).cuda()
    L = float(torch.sum((Wt * Zt) ** 2))
    dZt = 2.0 * Wt ** 2 * Zt
    dlam, dMt = B.dfc_lrr_backward(dZt, m=p.m)
    return L, B.from_device_colmajor(Zt), dlam, B.from_device_colmajor(dMt), info


def _loss_gpu(B, torch, M, lam, p, W, opts):
    Mt = B.to_device_colmajor(M)
    Zt, _, _ = B.dfc_lrr_solve(Mt, lam, p.perm, p.offsets, opts=opts, want_S=False)
    Wt = torch.from_numpy(np.ascontiguousarray(W.T)).cuda()
    return float(torch.sum((Wt * Zt) ** 2))


@pytest.mark.parametrize("seed,t,iters,every", [(31, 3, 25, 7), (32, 1, 20, 20), (33, 4, 30, 8)])
def test_backward_matches_oracle_gradient(seed, t, iters, every):
    import oracle
    from oracle import adjoint as adj
    from paper_1304_5583_amd import binding as B
    from paper_1304_5583_amd.datagen import small_problem
    torch = need_gpu()
    p = small_problem(seed, m=24, k=3, r=2, ns=12, n_replace=3, t=t, lam=0.4)
    rng = np.random.default_rng(seed)
    W = rng.uniform(0.0, 1.0, (p.n, p.n))
    fast = dict(mu0=0.05, rho=1.25)
    say(f"[adjoint s{seed}] m={p.m} n={p.n} t={p.t} iters={iters} every={every}")
    L, Z, dlam, dM, info = _gpu_grad(B, torch, p, W, _opts(B, iters, every, **fast))
    oo = oracle.ALMOptions(mu0=0.05, rho=1.25, fixed_iters=iters)
    with one_thread():
        # dL/dZ needs Z: the forward first, then the reverse sweep with 2 W^2 o Z
        tapes = []
        for i in range(p.t):
            cols = p.perm[p.offsets[i]:p.offsets[i + 1]]
            tapes.append(adj.unrolled_forward(p.M[:, cols], p.M, p.lam, oo))
        Zo = adj.dfc_combine(tapes, p.perm)[0]
        _, dMo, dlo = adj.dfc_forward_backward(p.M, p.lam, p.perm, p.offsets, oo, 2.0 * W ** 2 * Zo)
    ez, em = rel(Z, Zo), rel(dM, dMo)
    el = abs(dlam - dlo) / max(abs(dlo), 1e-300)
    say(f"  relZ={ez:.2e} rel dM={em:.2e} dlam gpu={dlam:.6e} oracle={dlo:.6e} rel={el:.2e} rank={info.rank.tolist()}")
    assert ez <= 1e-9
    assert em <= 1e-7 and el <= 1e-7
    assert np.abs(dMo).max() > 0


def test_backward_matches_finite_differences_on_gpu():
    from paper_1304_5583_amd import binding as B
    from paper_1304_5583_amd.datagen import small_problem
    torch = need_gpu()
    p = small_problem(34, m=30, k=3, r=3, ns=14, n_replace=4, t=3, lam=0.35)
    rng = np.random.default_rng(34)
    W = rng.uniform(0.0, 1.0, (p.n, p.n))
    fast = dict(mu0=0.05, rho=1.25)
    L, Z, dlam, dM, info = _gpu_grad(B, torch, p, W, _opts(B, 30, 10, **fast))
    plain = B.lrr_opts_default(fixed_iters=30, **fast)
    h = 1e-6
    fd = (_loss_gpu(B, torch, p.M, p.lam + h, p, W, plain) - _loss_gpu(B, torch, p.M, p.lam - h, p, W, plain)) / (2 * h)
    say(f"[adjoint FD] dlam={dlam:.8e} fd={fd:.8e}")
    assert abs(fd - dlam) <= 1e-5 * (abs(fd) + 1e-3)
    for t in range(2):
        D = rng.standard_normal(p.M.shape)
        fdm = (_loss_gpu(B, torch, p.M + h * D, p.lam, p, W, plain) -
               _loss_gpu(B, torch, p.M - h * D, p.lam, p, W, plain)) / (2 * h)
        ad = float(np.sum(dM * D))
        say(f"  direction {t}: <dM, D>={ad:.8e} fd={fdm:.8e}")
        assert abs(fdm - ad) <= 1e-5 * (abs(fdm) + 1e-3)


def test_backward_errors():
    from paper_1304_5583_amd import binding as B
    from paper_1304_5583_amd.datagen import small_problem
    torch = need_gpu()
    p = small_problem(35, m=16, k=2, r=2, ns=8, n_replace=2, t=2, lam=0.4)
    Mt = B.to_device_colmajor(p.M)
    ctx = B.Context(0)
    # no recorded forward
    dZ = torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda")
    with pytest.raises(B.LRRError) as e:
        B.dfc_lrr_backward(dZ, ctx=ctx, m=p.m)
    assert e.value.status == B.LRR_ENOTAPE
    # recording needs the unrolled map
    with pytest.raises(B.LRRError) as e:
        B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, opts=B.lrr_opts_default(save_for_backward=1), ctx=ctx)
    assert e.value.status == B.LRR_EINVAL
    # a later solve invalidates the record
    B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, opts=_opts(B, 10, 5), ctx=ctx)
    B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, opts=B.lrr_opts_default(fixed_iters=5), ctx=ctx)
    with pytest.raises(B.LRRError) as e:
        B.dfc_lrr_backward(dZ, ctx=ctx, m=p.m)
    assert e.value.status == B.LRR_ENOTAPE


def test_autograd_function_gradients():
    from paper_1304_5583_amd import binding as B
    from paper_1304_5583_amd.autograd import dfc_lrr
    from paper_1304_5583_amd.datagen import small_problem
    torch = need_gpu()
    p = small_problem(36, m=20, k=2, r=2, ns=10, n_replace=2, t=2, lam=0.4)
    Mt = B.to_device_colmajor(p.M).requires_grad_(True)
    lam = torch.tensor(p.lam, dtype=torch.float64, device="cuda", requires_grad=True)
    W = torch.rand((p.n, p.n), dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    opts = B.lrr_opts_default(fixed_iters=20, checkpoint_every=6, mu0=0.05, rho=1.25)
    Zt = dfc_lrr(Mt, lam, p.perm, p.offsets, opts)
    L = torch.sum((W * Zt) ** 2)
    gM, gl = torch.autograd.grad(L, (Mt, lam))
    # the same gradient through the C ABI directly
    Zt2, _, _ = B.dfc_lrr_solve(Mt.detach(), p.lam, p.perm, p.offsets,
                                opts=B.lrr_opts_default(fixed_iters=20, checkpoint_every=6, mu0=0.05, rho=1.25,
                                                        save_for_backward=1), want_S=False)
    dl, dMt = B.dfc_lrr_backward(2.0 * W ** 2 * Zt2, m=p.m)
    assert torch.equal(Zt.detach(), Zt2)
    assert torch.allclose(gM, dMt, rtol=0, atol=1e-12 * float(dMt.abs().max()))
    assert abs(float(gl) - dl) <= 1e-12 * abs(dl)
