"""Pins of the oracle's principal component analysis (Sec. 6, eqs. SNPCA,
NewObs, SNperEign, CumulSN): eigenvalues over tens of decades against a
60-digit Jacobi reference and against exact block spectra, and the sum rule
and reconstruction on the covariance of the method."""
import decimal

import numpy as np
import pytest

import oracle
import synth


def _jacobi_60_digits(C, sweeps=40):
    """Eigenvalues of a small symmetric matrix by cyclic two-sided Jacobi in
    60-digit decimal arithmetic (the reference for the FP64 results)."""
    D = decimal.Decimal
    with decimal.localcontext() as ctx:
        ctx.prec = 60
        n = len(C)
        A = [[D(repr(float(C[i][j]))) for j in range(n)] for i in range(n)]
        tol = D(10) ** -50
        for _ in range(sweeps):
            off = D(0)
            for p in range(n - 1):
                for q in range(p + 1, n):
                    apq = A[p][q]
                    if apq == 0:
                        continue
                    r = abs(apq) / (A[p][p] * A[q][q]).sqrt()
                    off = max(off, r)
                    if r < tol:
                        continue
                    th = (A[q][q] - A[p][p]) / (2 * apq)
                    t = (1 if th >= 0 else -1) / (abs(th) + (1 + th * th).sqrt())
                    c = 1 / (1 + t * t).sqrt()
                    s = c * t
                    for k in range(n):
                        akp, akq = A[k][p], A[k][q]
                        A[k][p], A[k][q] = c * akp - s * akq, s * akp + c * akq
                    for k in range(n):
                        apk, aqk = A[p][k], A[q][k]
                        A[p][k], A[q][k] = c * apk - s * aqk, s * apk + c * aqk
            if off < tol:
                break
        return np.array(sorted(float(A[i][i]) for i in range(n)))


@pytest.mark.parametrize("seed", [3, 7])
def test_graded_eigenvalues_vs_high_precision(seed):
    """A dense SPD matrix graded over 30 decades: every eigenvalue to 1e-12
    relative of the 60-digit reference; a plain symmetric eigensolver misses
    the small ones entirely."""
    rng = np.random.default_rng(seed)
    n = 14
    X = rng.normal(size=(n, n))
    A = X @ X.T / n + 0.05 * np.eye(n)
    s = 10.0 ** np.linspace(-15, 0, n)
    rng.shuffle(s)
    C = A * np.outer(s, s)
    ref = _jacobi_60_digits(C)
    lam, _, _ = oracle.Oracle.pca(C, np.ones(n), vectors=False)
    assert np.max(np.abs(lam / ref - 1.0)) < 1e-12
    assert np.max(np.abs(np.sort(np.linalg.eigvalsh(C)) / ref - 1.0)) > 1e-3


def test_block_spectrum_exact():
    """Permuted 2 x 2 blocks s (1, rho; rho, 1) with s over 30 decades:
    eigenvalues s (1 +- rho) and eigenvectors (1, +-1) / sqrt(2) on each pair,
    exactly."""
    rng = np.random.default_rng(5)
    m = 12
    s = 10.0 ** rng.uniform(-40, -10, m)
    rho = rng.uniform(-0.9, 0.9, m)
    n = 2 * m
    C = np.zeros((n, n))
    for k in range(m):
        C[2 * k, 2 * k] = C[2 * k + 1, 2 * k + 1] = s[k]
        C[2 * k, 2 * k + 1] = C[2 * k + 1, 2 * k] = s[k] * rho[k]
    P = rng.permutation(n)
    C = C[np.ix_(P, P)]
    lam, _, _, S = oracle.Oracle.pca(C, np.ones(n))
    assert np.max(np.abs(lam / np.sort(np.concatenate([s * (1 + rho), s * (1 - rho)])) - 1.0)) < 1e-14
    for a in range(n):  # position i of C holds the original index P[i]
        nz = np.flatnonzero(np.abs(S[a]) > 1e-12)
        assert len(nz) == 2 and P[nz[0]] // 2 == P[nz[1]] // 2
        assert np.allclose(np.abs(S[a, nz]), np.sqrt(0.5), rtol=1e-13, atol=0)


@pytest.fixture(scope="module")
def tiny_cov():
    o = oracle.Oracle(synth.make_tables("tiny"))
    return o.run()


def test_sum_rule_and_reconstruction(tiny_cov):
    """Sum over modes of (S/N)^2_a = d^T C^-1 d; S orthonormal; S^T diag(lambda)
    S = C to 1e-12 on the scale of sqrt(C_aa C_bb); the cumulative curve ends
    at the total and its increments fall."""
    C, d = tiny_cov["C"], tiny_cov["d"]
    lam, snr2, cum, S = oracle.Oracle.pca(C, d)
    assert np.all(lam > 0) and np.all(np.diff(lam) >= 0)
    assert abs(np.sum(snr2) - tiny_cov["snr2"]) < 1e-10 * tiny_cov["snr2"]
    assert abs(cum[-1] - tiny_cov["snr2"]) < 1e-10 * tiny_cov["snr2"]
    assert np.all(np.diff(cum, 2) <= 1e-12 * cum[-1])
    assert np.max(np.abs(S @ S.T - np.eye(len(d)))) < 1e-12
    sc = np.sqrt(np.diag(C))
    R = (S.T * lam) @ S
    assert np.max(np.abs(R - C) / np.outer(sc, sc)) < 1e-12
    # the largest eigenvalues are within reach of a plain eigensolver
    ev = np.linalg.eigvalsh(C)
    big = ev > 1e-8 * ev[-1]
    assert np.allclose(lam[big], ev[big], rtol=1e-8, atol=0)
    assert lam[-1] / lam[0] > 1e10
