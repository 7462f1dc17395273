"""Kernel-level GPU checks through the diagnostic C-ABI entry points.

Each building block is compared with a plain float64 reference on the same
inputs: the MFMA GEMM (all transpose cases, ragged edges, grids of more than
a thousand tiles), the blocked
Cholesky-based inverse of I + A A^T, and the batched block-Jacobi eigensolver
(uneven orders, clusters, rank deficiency)."""
import numpy as np
import pytest

from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("M,N,K", [(64, 64, 16), (77, 131, 45), (1, 5, 3), (200, 9, 300),
                                   (2111, 2061, 37), (1030, 4100, 21)])
def test_dgemm_matches_float64(ta, tb, M, N, K):
    _check_dgemm(ta, tb, M, N, K, (3, 1, 2))


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("M,N,K", [(128, 96, 100), (96, 128, 64), (512, 512, 500), (130, 70, 16), (70, 130, 32),
                                   (65, 65, 48), (64, 64, 1)])
def test_dgemm_even_leading_dimensions(ta, tb, M, N, K):
    """Even leading dimensions, ragged M / N edges and K of one, two and three
    16-deep tiles (the loop multiplies tiles in pairs, an odd last one alone,
    and loads two tiles ahead: past the end the loads must read zeros)."""
    _check_dgemm(ta, tb, M, N, K, (4, 2, 2))


@pytest.mark.parametrize("ta", [0, 1])
def test_dgemm_largest_leading_dimension(ta):
    """lda = 2^22 - 1, the largest the FP64 GEMM accepts (a K-tile's panel is
    addressed with 32-bit byte offsets; with op(A) = A^T the 64 rows of a tile
    span 63 lda): the product is right; lda = 2^22 is LRR_EINVAL."""
    torch = need_gpu()
    from paper_1304_5583_amd import binding as B
    M, N, K = 64, 8, 20
    lda = (1 << 22) - 1
    rng = np.random.default_rng(22)
    opA, opB = rng.standard_normal((M, K)), rng.standard_normal((K, N))
    stored = opA.T if ta else opA                      # K x M or M x K, column-major
    dA = torch.zeros((stored.shape[1], lda), dtype=torch.float64, device="cuda")
    dA[:, :stored.shape[0]] = torch.from_numpy(np.ascontiguousarray(stored.T)).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(opB.T)).cuda()
    dC = torch.zeros((N, M), dtype=torch.float64, device="cuda")
    B.lrr_diag_dgemm(bool(ta), False, dA, dB, dC, M, N, K, lda, K, M)
    ref = opA @ opB
    assert np.abs(dC.cpu().numpy().T - ref).max() <= 1e-13 * (1 + np.abs(ref).max()) * K
    with pytest.raises(B.LRRError) as e:
        B.lrr_diag_dgemm(bool(ta), False, dA, dB, dC, M, N, K, lda + 1, K, M)
    assert e.value.status == B.LRR_EINVAL
    del dA


def _check_dgemm(ta, tb, M, N, K, pads):
    torch = need_gpu()
    from paper_1304_5583_amd import binding as B
    say(f"dgemm ta={ta} tb={tb} M={M} N={N} K={K} pads={pads}")
    rng = np.random.default_rng(M * 1000 + N + K)
    opA = rng.standard_normal((M, K))
    opB = rng.standard_normal((K, N))
    C0 = rng.standard_normal((M, N))
    A = opA.T if ta else opA          # stored matrix (column-major)
    Bm = opB.T if tb else opB
    lda, ldb, ldc = A.shape[0] + pads[0], Bm.shape[0] + pads[1], M + pads[2]
    def dev(X, ld):
        P = np.zeros((ld, X.shape[1]))
        P[:X.shape[0]] = X
        return torch.from_numpy(np.ascontiguousarray(P.T)).cuda()
    dA, dB, dC = dev(A, lda), dev(Bm, ldb), dev(C0, ldc)
    B.lrr_diag_dgemm(bool(ta), bool(tb), dA, dB, dC, M, N, K, lda, ldb, ldc, alpha=0.75, beta=-0.5)
    got = dC.cpu().numpy().T[:M]
    ref = 0.75 * opA @ opB - 0.5 * C0
    assert np.abs(got - ref).max() <= 1e-13 * (1 + np.abs(ref).max()) * K
    # padding rows of C untouched
    assert np.array_equal(dC.cpu().numpy().T[M:], np.zeros((ldc - M, N)))


@pytest.mark.parametrize("N,K,ld", [(512, 500, 512), (600, 333, 602), (130, 64, 131), (1000, 17, 1001),
                                    (1500, 40, 1500)])
def test_symmetric_product_is_bitwise_the_full_product(N, K, ld):
    """C = A^T A through the symmetric kernel (tiles on and above the diagonal,
    mirrored) equals, bit for bit, the full-tile kernel's product of A^T with a
    separate copy of A (which takes the general path), and that full product is
    itself exactly symmetric; beta = 0 never reads C (NaN-filled)."""
    torch = need_gpu()
    from paper_1304_5583_amd import binding as B
    rng = np.random.default_rng(N + K)
    A = np.zeros((ld, N))
    A[:K] = rng.standard_normal((K, N))
    dA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    dA2 = dA.clone()
    C1 = torch.full((N, N), float("nan"), dtype=torch.float64, device="cuda")
    C2 = torch.full((N, N), float("nan"), dtype=torch.float64, device="cuda")
    B.lrr_diag_dgemm(True, False, dA, dA, C1, N, N, K, ld, ld, N, alpha=1.0, beta=0.0)
    B.lrr_diag_dgemm(True, False, dA, dA2, C2, N, N, K, ld, ld, N, alpha=1.0, beta=0.0)
    c1, c2 = C1.cpu().numpy().T, C2.cpu().numpy().T
    say(f"sym N={N} K={K}: max |sym - full| = {np.abs(c1 - c2).max():.3e}, asym of full = {np.abs(c2 - c2.T).max():.3e}")
    assert np.array_equal(c2, c2.T)
    assert np.array_equal(c1, c2)
    ref = A[:K].T @ A[:K]
    assert np.abs(c1 - ref).max() <= 1e-13 * (1 + np.abs(ref).max()) * K


@pytest.mark.parametrize("m,n", [(32, 40), (77, 120), (100, 200), (257, 300)])
def test_spd_inverse(m, n):
    torch = need_gpu()
    from paper_1304_5583_amd import binding as B
    say(f"spd_inverse m={m} n={n}")
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n)) / np.sqrt(n) * 3.0
    K = np.eye(m) + A @ A.T
    Kinv = B.lrr_diag_spd_inverse(B.to_device_colmajor(A)).cpu().numpy()
    ref = np.linalg.inv(K)
    cond = np.linalg.cond(K)
    assert np.abs(Kinv - ref).max() <= 1e-14 * cond * np.abs(ref).max() * m
    assert np.abs(K @ Kinv - np.eye(m)).max() <= 1e-13 * cond


@pytest.mark.parametrize("eig_block", [16, 32])
def test_syevj_batched_uneven(eig_block):
    torch = need_gpu()
    from paper_1304_5583_amd import binding as B
    rng = np.random.default_rng(eig_block)
    orders = [40, 100, 77, 3]
    ld = 100
    mats = []
    # PSD Gram, rank-deficient Gram, a matrix with a 5-fold repeated eigenvalue, tiny
    Y = rng.standard_normal((150, 40))
    mats.append(Y.T @ Y)
    Y = rng.standard_normal((100, 30)) @ rng.standard_normal((30, 100))
    mats.append(Y.T @ Y)
    Q, _ = np.linalg.qr(rng.standard_normal((77, 77)))
    ev = np.concatenate([np.full(5, 2.0), rng.uniform(0, 10, 72)])
    mats.append((Q * ev) @ Q.T)
    mats.append(np.array([[2.0, 1.0, 0.0], [1.0, 2.0, 0.0], [0.0, 0.0, 1.0]]))
    Bs = np.zeros((len(orders), ld, ld))
    for i, Mx in enumerate(mats):
        Mx = 0.5 * (Mx + Mx.T)
        mats[i] = Mx
        Bs[i, :orders[i], :orders[i]] = Mx
    say(f"syevj eig_block={eig_block} orders={orders}")
    lam, W, sweeps = B.lrr_diag_syevj(torch.from_numpy(Bs).cuda(), orders, eig_block=eig_block)
    lam, W = lam.cpu().numpy(), W.cpu().numpy()
    say(f"  sweeps={sweeps}")
    assert sweeps < 40
    for i, l in enumerate(orders):
        Wi = W[i].T[:l, :l]               # column-major storage -> columns are eigenvectors
        li = lam[i, :l]
        Mx = mats[i]
        nrm = np.abs(Mx).max()
        assert np.abs(Wi.T @ Wi - np.eye(l)).max() <= 1e-13 * l
        assert np.abs((Wi * li) @ Wi.T - Mx).max() <= 1e-13 * nrm * l
        ref = np.linalg.eigvalsh(Mx)
        assert np.abs(np.sort(li) - ref).max() <= 1e-13 * nrm * l


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("M,N,K", [(64, 64, 16), (77, 131, 45), (200, 9, 300), (130, 70, 1001)])
def test_reduced_precision_gemm_error_bound(prec, ta, tb, M, N, K):
    """FP32 and BF16x3 products against FP64 with the a-priori elementwise bound.

    FP32: each operand rounded once (u = 2^-24) and K-term FP32 accumulation,
    |C - AB| <= (K + 2) u (|A||B|).  BF16x3: x = hi + lo represents x to 2^-18
    relative, the dropped lo*lo term is below 2^-18 |a b|, and the 3K exact
    BF16 products are summed in FP32: |C - AB| <= (3 2^-18 + (3K + 2) u)(|A||B|).
    The product must also differ from the FP64 one (the reduced path ran)."""
    torch = need_gpu()
    from paper_1304_5583_amd import binding as B
    say(f"gemm prec={prec} ta={ta} tb={tb} M={M} N={N} K={K}")
    rng = np.random.default_rng(M * 7 + N * 3 + K + prec)
    opA = rng.standard_normal((M, K)) * np.exp(rng.uniform(-3, 3, (M, 1)))
    opB = rng.standard_normal((K, N))
    C0 = rng.standard_normal((M, N))
    A = opA.T if ta else opA
    Bm = opB.T if tb else opB
    dA, dB, dC = (torch.from_numpy(np.ascontiguousarray(X.T)).cuda() for X in (A, Bm, C0))
    B.lrr_diag_gemm(prec, bool(ta), bool(tb), dA, dB, dC, M, N, K, A.shape[0], Bm.shape[0], M,
                    alpha=0.75, beta=-0.5)
    got = dC.cpu().numpy().T
    ref = 0.75 * opA @ opB - 0.5 * C0
    scale = 0.75 * np.abs(opA) @ np.abs(opB)
    u = 2.0 ** -24
    bound = (K + 2) * u if prec == 1 else 3 * 2.0 ** -18 + (3 * K + 2) * u
    err = np.abs(got - ref)
    assert np.all(err <= bound * scale + 1e-15 * np.abs(ref))
    assert err.max() > 1e-13 * scale.max()


def test_reduced_precision_gemm_rejects_unknown_precision():
    torch = need_gpu()
    from paper_1304_5583_amd import binding as B
    X = torch.ones((4, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(B.LRRError) as e:
        B.lrr_diag_gemm(7, False, False, X, X, X, 4, 4, 4, 4, 4, 4)
    assert e.value.status == B.LRR_EINVAL
