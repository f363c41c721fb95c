"""Independent numpy replays of the oracle's decision rules (test helpers).

Each replay restates one rule of the method from its definition, with numpy and
scipy doing the arithmetic (dense solves, graph distances, sorting), so that it
shares nothing with the oracle's C code but the rule itself:

- aFSAI pattern growth (Section 3.1, Algorithm "aFSAI Smoother Set-up"): the
  FSAI row of a pattern from a dense solve of its local system, the gradient of
  the Kaporin-type functional on the candidate nodes, the top-rho choice and the
  eps_g stop of one row, and the outer loop over all rows;
- the theta filter of the strength-of-connection graph (Section 3.4);
- the interpolation candidates, C nodes within S-distance d_p (Section 3.5).

Decision quantities are compared after rounding to `bits` significant bits,
half to even (math.frexp / round / math.ldexp).
"""
from __future__ import annotations

import math

import numpy as np


def q(s, bits=20):
    """s rounded to `bits` significant bits, ties to even."""
    if s == 0.0:
        return 0.0
    m, e = math.frexp(s)
    return math.ldexp(round(m * 2 ** bits), e - bits)


def node_adjacency(rp, ci):
    """Node neighbour sets of a block pattern (self excluded)."""
    n = len(rp) - 1
    return [set(int(j) for j in ci[rp[i]:rp[i + 1]]) - {i} for i in range(n)]


def fsai_row(Ad, I, B, b=3):
    """Scalar rows of block row I for the off-diagonal node pattern B (ascending).

    For d = 0..b-1 the row solves its local system M_d x = e_last, M_d = A[l_d, l_d]
    with l_d = [(J,e) for J in B] + [(I,0..d)].  Returns (gp, psi, idx): gp[d] =
    x / x_last (unit last entry, the g' of the growth rule), psi[d] = 1 / x_last
    = min g^T A g over the pattern with g_last = 1, idx the scalar index list."""
    idx = [b * J + e for J in B for e in range(b)] + [b * I + e for e in range(b)]
    gp, psi = [], []
    for d in range(b):
        md = b * len(B) + d + 1
        li = idx[:md]
        rhs = np.zeros(md)
        rhs[-1] = 1.0
        x = np.linalg.solve(Ad[np.ix_(li, li)], rhs)
        gp.append(x / x[-1])
        psi.append(1.0 / x[-1])
    return gp, psi, idx


def fsai_scaled_rows(Ad, I, B, b=3):
    """The stored FSAI rows g = g' / sqrt(psi), so that diag(G A G^T) = 1."""
    gp, psi, idx = fsai_row(Ad, I, B, b)
    return [gp[d] / math.sqrt(psi[d]) for d in range(b)], idx


def growth_choice(Ad, adj, I, B, rho, b=3, bits=20):
    """One growth step of row I: the nodes J < I outside B adjacent to B u {I},
    scored by sum_d sum_e h^2 with h = A[(J,e), l_d] g'_d; the rho largest
    quantised scores > 0, ties to the lowest J.  Returns the added nodes."""
    cands = sorted({J for K in list(B) + [I] for J in adj[K] if J < I and J not in B})
    if not cands:
        return []
    gp, _, idx = fsai_row(Ad, I, B, b)
    scored = []
    for J in cands:
        s = 0.0
        for d in range(b):
            li = idx[:b * len(B) + d + 1]
            for e in range(b):
                h = Ad[b * J + e, li] @ gp[d]
                s += h * h
        if s > 0.0:
            scored.append((-q(s, bits), J))
    scored.sort()
    return [J for _, J in scored[:rho]]


def first_pass(Ad, adj, I, k_g, rho, eps_g, b=3, bits=20):
    """First pass of row I: from B = {} at most k_g growth steps; after a step
    the row stops when q(psi_prev - psi) <= q(eps_g psi_prev), psi the sum of
    the row's scalar psi, or when nothing was added.  Returns B (ascending)."""
    B = []
    psi_prev = sum(fsai_row(Ad, I, B, b)[1])
    for _ in range(k_g):
        add = growth_choice(Ad, adj, I, B, rho, b, bits)
        if not add:
            break
        B = sorted(B + add)
        psi = sum(fsai_row(Ad, I, B, b)[1])
        stop = q(psi_prev - psi, bits) <= q(eps_g * psi_prev, bits)
        psi_prev = psi
        if stop:
            break
    return B


def dense_G(Ad, patterns, b=3):
    """G from per-row patterns: full off-diagonal blocks, lower-triangular diagonal block."""
    n = len(patterns)
    G = np.zeros((n * b, n * b))
    for I, B in enumerate(patterns):
        rows, idx = fsai_scaled_rows(Ad, I, B, b)
        for d in range(b):
            li = idx[:b * len(B) + d + 1]
            G[b * I + d, li] = rows[d]
    return G


def outer_loop(Ad, adj, nnzb_A, k_g, rho, eps_g, omega_bar, b=3, bits=20, max_rounds=50):
    """The aFSAI outer loop: first passes, then while q(2 / lambda_1(G A G^T)) <
    q(omega_bar) and G has fewer blocks than A, every row takes one more growth
    step; stops also when a round changes no row.  lambda_1 from a dense
    symmetric eigensolve.  Returns (patterns, rounds, history of (nnzb(G), omega))."""
    n = len(adj)
    pats = [first_pass(Ad, adj, I, k_g, rho, eps_g, b, bits) for I in range(n)]
    rounds, hist = 0, []
    while rounds < max_rounds:
        G = dense_G(Ad, pats, b)
        lam = np.linalg.eigvalsh(G @ Ad @ G.T)[-1]
        nnzb_G = sum(len(B) + 1 for B in pats)
        hist.append((nnzb_G, 2.0 / lam))
        if not q(2.0 / lam, bits) < q(omega_bar, bits):
            break
        if not nnzb_G < nnzb_A:
            break
        changed = False
        new = []
        for I in range(n):
            add = growth_choice(Ad, adj, I, pats[I], rho, b, bits)
            changed |= bool(add)
            new.append(sorted(pats[I] + add))
        if not changed:
            break
        pats = new
        rounds += 1
    return pats, rounds, hist


def theta_filter(rp, ci, soc, theta, bits=20):
    """Strong graph from the SoC values on A's blocks: every node keeps its
    min(theta, deg) strongest connections with SoC > 0 (quantised, ties to the
    lowest J), then edges are symmetrised by union.  Returns neighbour sets."""
    n = len(rp) - 1
    keep = []
    for i in range(n):
        c = [(-q(soc[k], bits), int(ci[k])) for k in range(rp[i], rp[i + 1]) if soc[k] > 0.0]
        c.sort()
        keep.append({j for _, j in c[:theta]})
    S = [set() for _ in range(n)]
    for i in range(n):
        for j in keep[i]:
            S[i].add(j)
            S[j].add(i)
    return S


def soc_from_V(V, rp, ci, excluded):
    """Node affinity on A's off-diagonal blocks between non-excluded nodes:
    ||V_I V_J^T||_F^2 / (||V_I V_I^T||_F ||V_J V_J^T||_F) (0 where undefined)."""
    n = len(rp) - 1
    out = np.zeros(int(rp[-1]))
    nrm = [np.linalg.norm(V[i] @ V[i].T) for i in range(n)]
    for i in range(n):
        if excluded[i]:
            continue
        for k in range(rp[i], rp[i + 1]):
            j = int(ci[k])
            if j == i or excluded[j] or nrm[i] * nrm[j] == 0.0:
                continue
            out[k] = np.linalg.norm(V[i] @ V[j].T) ** 2 / (nrm[i] * nrm[j])
    return out


def candidates_within(S_rp, S_ci, cf, d_p):
    """C nodes at graph distance 1..d_p from each F node of the strong graph."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path
    n = len(S_rp) - 1
    M = sp.csr_matrix((np.ones(len(S_ci)), S_ci, S_rp), shape=(n, n))
    F = np.nonzero(cf == 0)[0]
    out = {}
    if F.size == 0:
        return out
    D = shortest_path(M, unweighted=True, indices=F)
    for r, i in enumerate(F):
        out[int(i)] = sorted(int(j) for j in np.nonzero((D[r] >= 1) & (D[r] <= d_p) & (cf == 1))[0])
    return out
