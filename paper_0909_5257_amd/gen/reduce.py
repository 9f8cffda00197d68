"""Exact reduction of the colour space the kernels accumulate in.

The paper accumulates J_alpha = sum_d c_{d alpha} A_d over its full basis
(eq. color-amplitude) and contracts J N J^* (eq. color-averaged-amplitude).
Two exact facts shrink the work without changing |M|^2:

1. J always lies in the row space of the diagram coefficient matrix C (D x K):
   for tree diagrams built from f^{abc} and T^a that space is much smaller
   than K for gluons (24 of 120 for six gluons, the (n-2)! count of the
   f-based structures).  With r independent rows R of C and pivot columns P
   (R[:, P] invertible), Bt = R[:, P]^{-1} R gives c_d = c_d[P] Bt for every
   diagram, so J = Bt^T J' with J' = J[P] and Q = J'^H (Bt N Bt^T) J'.
2. For the over-complete two-quark-line basis the colour matrix is singular:
   with S an independent subset of basis elements (kept greedily in basis
   order), every other element is T_b = sum_{a in S} R_ba T_a with
   R_b = N'[b, S] N'[S, S]^{-1} (exact, checked on the matrix), so the
   colour amplitude only needs y_S = J'_S + R^T J'_rest and Q = y^H N'[S, S] y.
   Diagram coefficient vectors stay sparse.

Everything is done in exact rational arithmetic; floating point is used only
to pick pivots, and the result is checked exactly on every diagram.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import scipy.linalg


def _inverse(m):
    """Exact inverse of a square Fraction matrix (Gauss-Jordan)."""
    n = len(m)
    a = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(m)]
    for col in range(n):
        piv = next(r for r in range(col, n) if a[r][col] != 0)
        a[col], a[piv] = a[piv], a[col]
        pv = a[col][col]
        a[col] = [x / pv for x in a[col]]
        for r in range(n):
            if r != col and a[r][col] != 0:
                f = a[r][col]
                a[r] = [x - f * y for x, y in zip(a[r], a[col])]
    return [row[n:] for row in a]


def _exact_matmul(a, b):
    """Exact product of two integer matrices (object arrays of Python ints).

    Uses int64 arithmetic when the bound max|a| * max|b| * inner cannot overflow it, and
    Python integers otherwise."""
    inner = a.shape[1]
    amax = max((abs(int(x)) for x in a.flat), default=0)
    bmax = max((abs(int(x)) for x in b.flat), default=0)
    if amax * bmax * max(inner, 1) < (1 << 62):
        return (a.astype(np.int64) @ b.astype(np.int64)).astype(object)
    return a.dot(b)


def _independent_columns(m, tol=1e-9):
    """Indices of a maximal set of linearly independent columns (float pivoting)."""
    arr = np.array([[float(x) for x in row] for row in m])
    if not arr.size:
        return []
    _, rr, piv = scipy.linalg.qr(arr, pivoting=True, mode="economic")
    d = np.abs(np.diag(rr))
    rank = int(np.sum(d > tol * d.max())) if d.size else 0
    return sorted(piv[:rank].tolist())


class ColourSpace:
    """Accumulation vectors per diagram and the matrix W with Q = y^H W y."""

    def __init__(self, dag, nmat):
        k = len(dag.basis)
        coefs = [a.coef for a in dag.amps]
        rows = {}
        for c in coefs:
            if c:
                key = tuple(sorted(c.items()))
                rows.setdefault(key, c)
        uniq = list(rows.values())
        cmat = np.zeros((len(uniq), k))
        for i, c in enumerate(uniq):
            for j, v in c.items():
                cmat[i, j] = v
        # 1. row space of the coefficient matrix
        row_sel = _independent_columns(cmat.T.tolist())
        r = len(row_sel)
        if r < k:
            assert np.array_equal(cmat, np.round(cmat)), "diagram colour coefficients must be integers"
            rint = cmat[row_sel].astype(np.int64)
            piv = _independent_columns(rint.tolist())
            assert len(piv) == r
            inv = _inverse([[Fraction(int(rint[i, j])) for j in piv] for i in range(r)])
            # Bt = inv R in integers: Bt = BtD / d with d the common denominator of inv
            d = 1
            for row in inv:
                for x in row:
                    d = d * x.denominator // math.gcd(d, x.denominator)
            inv_d = np.array([[int(x * d) for x in row] for row in inv], dtype=object)
            bt_d = _exact_matmul(inv_d, rint.astype(object))
            # exact check on every distinct diagram vector: d c = c[P] (d Bt)
            cint = cmat.astype(np.int64).astype(object)
            assert np.array_equal(cint * d, _exact_matmul(cint[:, piv], bt_d)), \
                "colour coefficient vector outside the row space"
            # N' = Bt N Bt^T with N = n_l / l
            l = 1
            for row in nmat:
                for x in row:
                    l = l * x.denominator // math.gcd(l, x.denominator)
            n_l = np.array([[int(x * l) for x in row] for row in nmat], dtype=object)
            neff_num = _exact_matmul(_exact_matmul(bt_d, n_l), bt_d.T)
            den = d * d * l
            neff = [[Fraction(int(neff_num[a, b]), den) for b in range(r)] for a in range(r)]
            self.pivots = piv
        else:
            neff = [list(row) for row in nmat]
            self.pivots = list(range(k))
        # 2. singular colour matrix: keep an independent subset S (greedy, in basis
        #    order) and substitute T_b = sum_{a in S} R_ba T_a for the others
        sel = _greedy_independent(neff)
        if len(sel) < len(neff):
            nss = [[neff[i][j] for j in sel] for i in sel]
            inv_ss = _inverse(nss)
            rest = [i for i in range(len(neff)) if i not in sel]
            rmat = {b: [sum(neff[b][sel[c]] * inv_ss[c][a] for c in range(len(sel))) for a in range(len(sel))]
                    for b in rest}
            # exact check: N'[b, :] = R_b N'[S, :] for every dependent b (so T_b = R_b T_S)
            for b in rest:
                for j in range(len(neff)):
                    assert neff[b][j] == sum(rmat[b][a] * neff[sel[a]][j] for a in range(len(sel))), \
                        "colour basis relation is not exact"
            self.subst = (sel, rmat)
            self.w = nss
        else:
            self.subst = None
            self.w = neff
        self.dim = len(self.w)
        self.k = k

    def vector(self, coef: dict) -> dict:
        """Accumulation coefficients of one diagram (index -> Fraction)."""
        jp = {a: Fraction(coef[p]) for a, p in enumerate(self.pivots) if coef.get(p, 0)}
        if self.subst is None:
            return jp
        sel, rmat = self.subst
        pos = {b: a for a, b in enumerate(sel)}
        out = {}
        for b, v in jp.items():
            if b in pos:
                out[pos[b]] = out.get(pos[b], 0) + v
            else:
                for a, r in enumerate(rmat[b]):
                    if r != 0:
                        out[a] = out.get(a, 0) + v * r
        return {a: v for a, v in out.items() if v != 0}


def _greedy_independent(m, tol=1e-9):
    """Indices kept in order when each is linearly independent of those before (float test)."""
    arr = np.array([[float(x) for x in row] for row in m])
    kept = []
    for b in range(len(arr)):
        trial = kept + [b]
        sub = arr[np.ix_(trial, trial)]
        if np.linalg.matrix_rank(sub, tol=tol * max(1.0, np.abs(arr).max())) == len(trial):
            kept.append(b)
    return kept
