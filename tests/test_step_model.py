"""CPU model of the preconditioner's block step (the Jacobi method of Algorithm 2 step 3,
taken on a block pair's Gram matrix): the rotations of a step applied two-sided to
G = X_b^T X_b, G <- J^T G J with the same pairs and angles, and accumulated in Q, must
give X_b Q equal to the one-sided rotations of the columns, and keep G equal to
(X_b Q)^T (X_b Q) and exactly symmetric.  Pins the partner-and-coefficient convention
of the GPU kernel (the partner of the first column of a pair enters with -sin, that of
the second with +sin); no GPU needed."""
import numpy as np
import pytest

JB = 16
JC = 2 * JB


def _cs(al, be, ga):
    # tan 2t = 2 ga / (be - al), |t| <= pi / 4; x' = c x - s y, y' = s x + c y
    d = be - al
    r = np.hypot(d, 2.0 * ga)
    c = np.sqrt(0.5 + 0.5 * abs(d) / r)
    s = ga / (r * c)
    return c, (-s if d < 0 else s)


def _rr_pair(r, g, m):
    return (r, m - 1) if g == 0 else ((r + g) % (m - 1), (r - g + (m - 1)) % (m - 1))


def _rounds(first):
    out = []
    if first:  # the pairs inside each block
        for r in range(JB - 1):
            prs = []
            for k in range(JB):
                h = k // (JB // 2)
                p, q = _rr_pair(r, k % (JB // 2), JB)
                prs.append((p + JB * h, q + JB * h))
            out.append(prs)
    for r in range(JB):  # the cross pairs
        out.append([(k, JB + (k + r) % JB) for k in range(JB)])
    return out


@pytest.mark.parametrize("first", [True, False])
def test_gram_step_matches_one_sided(first):
    rng = np.random.default_rng(7)
    X = rng.standard_normal((300, JC)) * np.logspace(0, -6, JC)  # graded columns
    tol2 = 2.0 ** -48
    Y = X.copy()
    for prs in _rounds(first):
        for p, q in prs:
            al, be, ga = Y[:, p] @ Y[:, p], Y[:, q] @ Y[:, q], Y[:, p] @ Y[:, q]
            if ga * ga > tol2 * al * be:
                c, s = _cs(al, be, ga)
                Y[:, p], Y[:, q] = c * Y[:, p] - s * Y[:, q], c * Y[:, q] + s * Y[:, p]
    G, Q = X.T @ X, np.eye(JC)
    for prs in _rounds(first):
        cr, tr, pr = np.ones(JC), np.zeros(JC), np.arange(JC)
        for p, q in prs:
            c, s = 1.0, 0.0
            if G[p, q] ** 2 > tol2 * G[p, p] * G[q, q]:
                c, s = _cs(G[p, p], G[q, q], G[p, q])
            cr[p], tr[p], pr[p] = c, -s, q
            cr[q], tr[q], pr[q] = c, s, p
        Gn = np.empty_like(G)
        for a in range(JC):
            for b in range(JC):
                a0, b0 = min(a, b), max(a, b)
                pa, pb = pr[a0], pr[b0]
                Gn[a, b] = (cr[a0] * cr[b0] * G[a0, b0] + cr[a0] * tr[b0] * G[a0, pb]
                            + tr[a0] * cr[b0] * G[pa, b0] + tr[a0] * tr[b0] * G[pa, pb])
        Q = Q * cr[None, :] + Q[:, pr] * tr[None, :]
        G = Gn
    Yg = X @ Q
    scale = np.abs(Y).max(axis=0)
    assert np.max(np.abs(Yg - Y).max(axis=0) / scale) < 1e-13
    assert np.array_equal(G, G.T)
    assert np.max(np.abs(G - Yg.T @ Yg)) < 1e-13 * np.abs(G).max()
