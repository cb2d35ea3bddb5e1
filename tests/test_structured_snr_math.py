"""The algebra behind the structured S/N, checked on the CPU with the
oracle's own matrices (no GPU code involved).

The joint covariance splits as C = C_G + E M E^T: C_G is the Gaussian term
(block-diagonal over ell-configurations, eqs. CovPPG and the Gaussian term of
App. B), E maps each data-vector row to its distinct row (the Limber kernels
are symmetric in the bins, so the values of d, the one-halo term and the
response depend only on the multiset of bins), and M = C_1h + sigma_b^2 r r^T
on the distinct rows.  Because also d = E d_R,
    (S/N)^2 = d^T C^-1 d = d_R^T (G^-1 + M)^-1 d_R,   G = E^T C_G^-1 E,
and with G = L L^T:  (S/N)^2 = u^T (I + Z)^-1 u,  u = L^T d_R,  Z = L^T M L.
Each block of G has a closed form in Q = (P^s)^-1 per ell-bin: on the pairs
i <= j, S2(P)^-1 = (nu nu^T / 4) o S2(Q), and on the triples i <= j <= k,
S3(P)^-1 = (mu mu^T / 36) o S3(Q), where S2 and S3 are the symmetrised
products of the Gaussian term and nu, mu count the distinct orderings."""
import itertools

import numpy as np
import pytest

import oracle
import synth


def _pairs(n):
    return [(i, j) for i in range(n) for j in range(i, n)]


def _trips(n):
    return [(i, j, k) for i in range(n) for j in range(i, n) for k in range(j, n)]


def _orderings(m):
    return sorted(set(itertools.permutations(m)))


def _S2(P, idx):
    return np.array([[P[i, a] * P[j, b] + P[i, b] * P[j, a] for (a, b) in idx] for (i, j) in idx])


def _S3(P, idx):
    out = np.zeros((len(idx), len(idx)))
    for x, m in enumerate(idx):
        for y, mp in enumerate(idx):
            out[x, y] = sum(P[m[0], s[0]] * P[m[1], s[1]] * P[m[2], s[2]] for s in itertools.permutations(mp))
    return out


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, n))
    return X @ X.T + n * np.eye(n)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_symmetrised_inverses(n):
    P = _spd(n, n)
    Q = np.linalg.inv(P)
    pr = _pairs(n)
    nu = np.array([len(_orderings(p)) for p in pr], float)
    assert np.allclose(np.linalg.inv(_S2(P, pr)), np.outer(nu, nu) / 4 * _S2(Q, pr), rtol=1e-10, atol=0)
    tr = _trips(n)
    mu = np.array([len(_orderings(t)) for t in tr], float)
    assert np.allclose(np.linalg.inv(_S3(P, tr)), np.outer(mu, mu) / 36 * _S3(Q, tr), rtol=1e-10, atol=0)


def _closed_form_G(o, reps, canon):
    """G = E^T C_G^-1 E block by block from the closed forms."""
    n = o.n_z
    ps = o.ps_table()          # [n_ell][n_z][n_z] P^s
    nm, nt = o.nmodes(), o.ntri()
    Q = np.array([np.linalg.inv(ps[b]) for b in range(o.n_ell)])
    rows = o.rows
    nR = len(reps)
    G = np.zeros((nR, nR))
    # rows of the data vector that map to each distinct row
    members = [[] for _ in range(nR)]
    for a, e in enumerate(canon):
        members[e].append(a)
    for e in range(nR):
        for f in range(nR):
            a0, b0 = reps[e], reps[f]
            if rows["cfg"][a0] != rows["cfg"][b0]:
                continue
            if rows["kind"][a0] == 2:
                b = rows["lbin"][a0][0]
                (i, j), (k, l) = rows["zbin"][a0][:2], rows["zbin"][b0][:2]
                nu = lambda x, y: 1.0 if x == y else 2.0
                G[e, f] = nm[b] * nu(i, j) * nu(k, l) / 4 * (Q[b][i, k] * Q[b][j, l] + Q[b][i, l] * Q[b][j, k])
                continue
            l1, l2, l3 = rows["lbin"][a0]
            kap = nt[rows["tri"][a0]] / o.omega  # inverse of Omega / N_tri
            val = 0.0
            for a in members[e]:
                for bb in members[f]:
                    z, zp = rows["zbin"][a], rows["zbin"][bb]
                    if l1 == l2 == l3:
                        m, mp = tuple(z), tuple(zp)
                        mu = len(_orderings(m)) * len(_orderings(mp))
                        val += mu / 36 * sum(Q[l1][m[0], s[0]] * Q[l1][m[1], s[1]] * Q[l1][m[2], s[2]]
                                              for s in itertools.permutations(mp))
                    elif l1 == l2:
                        nu = (1.0 if z[0] == z[1] else 2.0) * (1.0 if zp[0] == zp[1] else 2.0)
                        s2 = Q[l1][z[0], zp[0]] * Q[l1][z[1], zp[1]] + Q[l1][z[0], zp[1]] * Q[l1][z[1], zp[0]]
                        val += nu / 4 * s2 * Q[l3][z[2], zp[2]]
                    elif l2 == l3:
                        nu = (1.0 if z[1] == z[2] else 2.0) * (1.0 if zp[1] == zp[2] else 2.0)
                        s2 = Q[l2][z[1], zp[1]] * Q[l2][z[2], zp[2]] + Q[l2][z[1], zp[2]] * Q[l2][z[2], zp[1]]
                        val += nu / 4 * s2 * Q[l1][z[0], zp[0]]
                    else:
                        val += Q[l1][z[0], zp[0]] * Q[l2][z[1], zp[1]] * Q[l3][z[2], zp[2]]
            G[e, f] = kap * val
    return G


@pytest.mark.parametrize("preset,tomo", [("tiny", "paper"), ("tiny", "sorted"), ("mid", "paper")])
def test_structured_snr_identity(preset, tomo):
    t = synth.make_tables(preset)
    o = oracle.Oracle(t, tomo=tomo)
    d, r = o.data_vector()
    N = o.N
    canon, reps = oracle.canonical_rows(o.rows)
    canon = np.asarray(canon)
    reps = np.asarray(reps)
    nR = len(reps)
    E = np.zeros((N, nR))
    E[np.arange(N), canon] = 1.0
    d_R, r_R = d[reps], r[reps]
    assert np.array_equal(E @ d_R, d) and np.array_equal(E @ r_R, r)
    ii, jj = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    CG = o.gauss_pairs(np.stack([ii.ravel(), jj.ravel()], 1)).reshape(N, N)
    ei, ej = np.meshgrid(reps, reps, indexing="ij")
    M = o.cov1h_pairs(np.stack([ei.ravel(), ej.ravel()], 1)).reshape(nR, nR) + \
        float(t.cfg["sigma_b2"]) * np.outer(r_R, r_R)
    direct = oracle.Oracle.snr2(CG + E @ M @ E.T, d)
    G = E.T @ np.linalg.solve(CG, E)
    if tomo == "paper":
        # the PAPER rows of each configuration form a product set over the
        # legs, so the Gaussian block is a (symmetrised) Kronecker product;
        # with SORTED rows E = I and the structured form is the plain one
        Gc = _closed_form_G(o, reps, canon)
        for e in range(nR):  # block by block, relative to the block's scale
            blk = o.rows["cfg"][reps] == o.rows["cfg"][reps[e]]
            assert np.max(np.abs(Gc[e, blk] - G[e, blk])) <= 1e-10 * np.max(np.abs(G[e, blk]))
        G = Gc
    L = np.linalg.cholesky(G)
    u = L.T @ d_R
    Z = L.T @ M @ L
    structured = float(u @ np.linalg.solve(np.eye(nR) + Z, u))
    assert abs(structured - direct) <= 1e-10 * direct
