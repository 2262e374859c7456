"""Test-side constructions taken directly from the paper's definitions.

These are written independently of the oracle's loop code: the constraint
matrix comes from the Kronecker products of def:A1A2A3 / def:A4, and the full
OT LP from eq. model:OT.  They pin the oracle, they do not share code with it.
"""
import numpy as np


def kron_A(m, n):
    """Dense A of eq. Mat:A&b from the Kronecker forms (def:A1A2A3, def:A4)."""
    M = m * n
    Im, In, IM = np.eye(m), np.eye(n), np.eye(M)
    one_m, one_n = np.ones((1, m)), np.ones((1, n))
    A1 = np.kron(IM, one_m)                      # M x m^2 n
    A2 = -np.kron(one_n, IM)                     # M x m n^2
    A3 = np.kron(In, np.kron(one_m, Im))         # M x m^2 n
    A4hat = np.kron(In, np.kron(one_n, Im))      # M x m n^2
    A4 = A4hat[:-1]                              # Ibar on the last block drops its last row
    top = np.hstack([A1, A2])
    mid = np.hstack([A3, np.zeros((M, m * n * n))])
    bot = np.hstack([np.zeros((M - 1, m * m * n)), A4])
    return np.vstack([top, mid, bot])


def aat_blocks(m, n):
    """A A^T assembled from the blocks E1..E5 of eq. Mat:OT_AAT."""
    M = m * n
    E1 = (m + n) * np.eye(M)
    E2 = np.kron(np.eye(n), np.ones((m, m)))
    Ibar = np.eye(m)[:-1]                        # (m-1) x m
    row = np.hstack([np.eye(m)] * (n - 1) + [Ibar.T])   # m x (M-1)
    E3 = -np.kron(np.ones((n, 1)), row)          # M x (M-1)
    E4 = m * np.eye(M)
    E5 = n * np.eye(M - 1)
    Z = np.zeros((M, M - 1))
    return np.block([[E1, E2, E3], [E2.T, E4, Z], [E3.T, Z.T, E5]])


def full_ot_lp(mu1, mu2):
    """Eq. model:OT: variables pi[(i,j),(k,l)], row-major over source then target."""
    m, n = mu1.shape
    M = m * n
    bins = [(i, j) for i in range(m) for j in range(n)]
    c = np.array([(i - k) ** 2 + (j - l) ** 2 for (i, j) in bins for (k, l) in bins], float)
    Aeq = np.zeros((2 * M, M * M))
    for s in range(M):
        Aeq[s, s * M:(s + 1) * M] = 1.0          # sum over targets = mu1
    for t in range(M):
        Aeq[M + t, t::M] = 1.0                   # sum over sources = mu2
    beq = np.concatenate([mu1.ravel(), mu2.ravel()])
    return Aeq, beq, c


def reduced_lp(mu1, mu2, oracle):
    m, n = mu1.shape
    return kron_A(m, n), oracle.bvec(mu1, mu2), oracle.cost(m, n)


def highs(Aeq, beq, c):
    from scipy.optimize import linprog
    r = linprog(c, A_eq=Aeq, b_eq=beq, bounds=(0, None), method="highs")
    assert r.status == 0, r.message
    return r.fun, r.x


def rand_hist(rng, m, n, zeros=0.0):
    h = rng.uniform(0.05, 1.0, size=(m, n))
    if zeros:
        h[rng.uniform(size=(m, n)) < zeros] = 0.0
        if h.sum() == 0:
            h[0, 0] = 1.0
    return h / h.sum()


def full_ot_lp_xy(mu1, mu2, u, v):
    """Eq. model:OT on a grid whose row i sits at u[i] and column j at v[j]:
    cost (u_i - u_k)^2 + (v_j - v_l)^2 between bins (i,j) and (k,l)."""
    m, n = mu1.shape
    pos = np.array([(u[i], v[j]) for i in range(m) for j in range(n)])
    diff = pos[:, None, :] - pos[None, :, :]
    c = (diff ** 2).sum(-1).ravel()
    Aeq, beq, _ = full_ot_lp(mu1, mu2)
    return Aeq, beq, c


def w2_1d_positions(a, b, x):
    """1-D W2^2 between masses a and b at sorted positions x: the quantile
    coupling pairs the overlap of [A_{p-1}, A_p) and [B_{q-1}, B_q)."""
    A, B = np.concatenate([[0], np.cumsum(a)]), np.concatenate([[0], np.cumsum(b)])
    tot = 0.0
    for p in range(len(a)):
        for q in range(len(b)):
            ov = min(A[p + 1], B[q + 1]) - max(A[p], B[q])
            if ov > 0:
                tot += ov * (x[p] - x[q]) ** 2
    return tot
