"""Colour basis, diagram colour factors and the colour matrix (oracle).

All colour objects are evaluated numerically on explicit colour assignments:
one index per external leg (0..7 for a gluon, 0..2 for a quark leg).

* Basis (section 2.1, eq. color-amplitude; eq. color-basis for gluons; counts
  in Table 1):
    - all gluons: T_alpha = Tr(t^{c_0} t^{c_s1} ... t^{c_s(n-1)}), one entry per
      ordering s of legs 1..n-1 with leg 0 held first, (n-1)! in all;
    - one quark line from 'qi' leg j to 'qo' leg i: T_alpha =
      (t^{c_s1} ... t^{c_sk})_{c_i c_j}, one entry per ordering of the k
      gluons, k! in all;
    - two quark lines: for each of the two ways of joining the two 'qi' legs
      to the two 'qo' legs, T_alpha = sum_x (W_1)_{c_i1 c_j1} (W_2)_{c_i2 c_j2}
      where the words W_1, W_2 each hold the summed adjoint index x once and
      the external gluons are shared out between them in order.
* Diagram colour factor C_d(c): the product of the Feynman-rule colour
  factors f^{abc} (three-gluon), f f (each four-gluon piece) and t^a_{ij}
  (quark-gluon), contracted along the diagram's internal lines.
* Decomposition: C_d(c) = sum_alpha c_{d alpha} T_alpha(c) for all c, solved by
  least squares on a random set of assignments that reaches the full rank of
  the basis, and checked on a second independent set.
* Colour matrix (eq. color-matrix): N_{alpha beta} =
  1/(n_a n_b) sum_c T_alpha(c) T_beta(c)^*, summed over every assignment.
"""
from __future__ import annotations

import functools
import itertools
from fractions import Fraction

import numpy as np

from .process import OracleProcess, enumerate_diagrams, fermion_sign, parse_process
from .su3 import F, T

BRIDGE = "x"   # name of the shared adjoint index of the two-line basis


def colour_basis(proc: OracleProcess) -> list:
    """Basis descriptors.

    Each descriptor is a tuple of strands (row_leg, col_leg, word); a trace
    is written with row_leg = col_leg = None.  Words are tuples of gluon legs
    and possibly BRIDGE.
    """
    kinds = proc.kinds
    gluons = [i for i, k in enumerate(kinds) if k == "g"]
    qi = [i for i, k in enumerate(kinds) if k == "qi"]
    qo = [i for i, k in enumerate(kinds) if k == "qo"]
    basis = []
    if not qi:
        first, rest = gluons[0], gluons[1:]
        for perm in itertools.permutations(rest):
            basis.append(((None, None, (first,) + perm),))
    elif len(qi) == 1:
        for perm in itertools.permutations(gluons):
            basis.append(((qo[0], qi[0], perm),))
    else:
        for pairing in (dict(zip(qi, qo)), dict(zip(qi, qo[::-1]))):
            for r in range(len(gluons) + 1):
                for g1 in itertools.combinations(gluons, r):
                    g2 = [g for g in gluons if g not in g1]
                    for w1 in itertools.permutations(list(g1) + [BRIDGE]):
                        for w2 in itertools.permutations(g2 + [BRIDGE]):
                            basis.append(((pairing[qi[0]], qi[0], w1),
                                          (pairing[qi[1]], qi[1], w2)))
    return basis


def _word_matrices(word, c, xval=None):
    """Product of t matrices along a word for every assignment row: [m,3,3]."""
    m = c.shape[0]
    out = np.broadcast_to(np.eye(3, dtype=np.complex128), (m, 3, 3)).copy()
    for letter in word:
        mat = T[xval] if letter == BRIDGE else T[c[:, letter]]
        out = out @ mat
    return out


def basis_values(proc: OracleProcess, basis: list, c: np.ndarray) -> np.ndarray:
    """T_alpha(c) for assignment rows c [m, n]: complex [m, K].

    Row by row: each strand is a product of explicit 3x3 matrices.
    """
    m = c.shape[0]
    rows = np.arange(m)
    out = np.empty((m, len(basis)), dtype=np.complex128)
    for a, desc in enumerate(basis):
        has_x = any(BRIDGE in s[2] for s in desc)
        xs = range(8) if has_x else [None]
        val = np.zeros(m, dtype=np.complex128)
        for x in xs:
            term = np.ones(m, dtype=np.complex128)
            for row_leg, col_leg, word in desc:
                mats = _word_matrices(word, c, x)
                if row_leg is None:
                    term = term * np.trace(mats, axis1=1, axis2=2)
                else:
                    term = term * mats[rows, c[:, row_leg], c[:, col_leg]]
            val += term
        out[:, a] = val
    return out


_LETTERS = "abcdefghijklmnopqrstuvwxyz"


@functools.lru_cache(maxsize=None)
def _chain_tensor(length: int) -> np.ndarray:
    """(t^{b1} ... t^{bL})_{ij} as a tensor [8]*L + [3, 3]."""
    w = np.eye(3, dtype=np.complex128)
    for _ in range(length):
        w = np.tensordot(w, T, axes=([-1], [1]))        # [..., i, b, k]
        w = np.moveaxis(w, -2, -3)                       # [..., b, i, k]
    # axes are now [b1, ..., bL, i, j] after the moves above
    return w


def basis_tensor_all(proc: OracleProcess, basis: list) -> np.ndarray:
    """T_alpha(c) for every colour assignment c, complex [prod(dims), K].

    Same values as basis_values on all_assignments (rows in that order), but
    each strand's matrix product is formed once as a full tensor over its
    letters and the legs are then read off by index relabelling.
    """
    n = proc.n
    leg_sym = {i: _LETTERS[i] for i in range(n)}
    out = []
    for desc in basis:
        operands, subs = [], []
        extra = iter(_LETTERS[n:])
        xsym = next(extra)
        for row_leg, col_leg, word in desc:
            letters = "".join(xsym if l == BRIDGE else leg_sym[l] for l in word)
            operands.append(_chain_tensor(len(word)))
            if row_leg is None:
                r = next(extra)
                subs.append(letters + r + r)
            else:
                subs.append(letters + leg_sym[row_leg] + leg_sym[col_leg])
        expr = ",".join(subs) + "->" + "".join(leg_sym[i] for i in range(n))
        out.append(np.einsum(expr, *operands, optimize=True).reshape(-1))
    return np.stack(out, axis=1)


def _f_ab(a, b):
    """sum_{a,b} f^{a b e} A_a B_b per row: [m, 8]."""
    x = (a @ F.reshape(8, 64)).reshape(-1, 8, 8)        # [m, b, e]
    return np.einsum("mbe,mb->me", x, b)


def _t_col(a, psi):
    """sum_{a,j} t^a_{i j} A_a psi_j per row: [m, 3]."""
    x = (a @ T.reshape(8, 9)).reshape(-1, 3, 3)
    return np.einsum("mij,mj->mi", x, psi)


def _t_row(psibar, a):
    """sum_{a,i} psibar_i t^a_{i j} A_a per row: [m, 3]."""
    x = (a @ T.reshape(8, 9)).reshape(-1, 3, 3)
    return np.einsum("mi,mij->mj", psibar, x)


def _t_adj(psibar, psi):
    """psibar_i t^a_{i j} psi_j per row: [m, 8]."""
    return np.einsum("mi,aij,mj->ma", psibar, T, psi, optimize=True)


def diagram_colour_values(tree, root_kind: str, proc: OracleProcess, c: np.ndarray) -> np.ndarray:
    """C_d(c) of one diagram at assignment rows c [m, n]: complex [m]."""
    m = c.shape[0]
    rows = np.arange(m)

    def onehot(leg, dim):
        v = np.zeros((m, dim), dtype=np.complex128)
        v[rows, c[:, leg]] = 1.0
        return v

    def ev(t):
        tag = t[0]
        if tag == "leg":
            leg = t[1]
            return onehot(leg, 8 if proc.kinds[leg] == "g" else 3)
        if tag == "ggg":
            return _f_ab(ev(t[1]), ev(t[2]))
        if tag == "gggg":
            k, a, b, cc = t[1], ev(t[2]), ev(t[3]), ev(t[4])
            if k == 0:      # f^{abe} f^{cde}: sum_{c,e} f^{c d e} C_c X_e
                return -_f_ab(cc, _f_ab(a, b))
            if k == 1:      # f^{ace} f^{bde}
                return -_f_ab(b, _f_ab(a, cc))
            return -_f_ab(a, _f_ab(b, cc))    # f^{ade} f^{bce}
        if tag == "qqg_i":          # t^a_{i j} psi_j
            return _t_col(ev(t[2]), ev(t[1]))
        if tag == "qqg_o":          # psibar_i t^a_{i j}
            return _t_row(ev(t[1]), ev(t[2]))
        if tag == "qq_g":           # psibar_i t^a_{i j} psi_j
            return _t_adj(ev(t[2]), ev(t[1]))
        raise AssertionError(tag)

    vec = ev(tree)
    return vec[rows, c[:, proc.root]]


def all_assignments(proc: OracleProcess) -> np.ndarray:
    dims = proc.colour_dims()
    grids = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    return np.stack([g.ravel() for g in grids], axis=1)


def random_assignments(proc: OracleProcess, m: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    dims = np.array(proc.colour_dims())
    return (rng.random((m, len(dims))) * dims).astype(np.int64)


def _rationalise(x: float, max_den: int = 1 << 20) -> Fraction:
    fr = Fraction(x).limit_denominator(max_den)
    if abs(float(fr) - x) > 1e-9 * max(1.0, abs(x)):
        raise ValueError(f"{x!r} is not a small rational")
    return fr


class ColourData:
    """Basis, colour matrix and decomposition coefficients of one process."""

    def __init__(self, spec: str):
        self.proc = parse_process(spec)
        self.diagrams = enumerate_diagrams(self.proc)
        self.signs = np.array([fermion_sign(t, self.proc) for t, _ in self.diagrams], dtype=np.float64)
        self.basis = colour_basis(self.proc)
        self._matrix()
        self._decompose()

    @property
    def n_colours(self) -> int:
        return len(self.basis)

    def _matrix(self):
        b = basis_tensor_all(self.proc, self.basis)
        acc = (b.T @ b.conj()) / self.proc.initial_colour_dof()
        assert np.max(np.abs(acc.imag)) < 1e-10 * max(1.0, np.max(np.abs(acc.real)))
        self.N_frac = [[_rationalise(v) for v in row] for row in acc.real]
        self.N = np.array([[float(v) for v in row] for row in self.N_frac])
        ev = np.linalg.eigvalsh(self.N)
        self.rank = int(np.sum(ev > 1e-9 * ev.max()))

    def _decompose(self):
        k, d = len(self.basis), len(self.diagrams)
        m = 8 * k + 1024
        seed = 20090930
        while True:
            c = random_assignments(self.proc, m, seed)
            b = basis_values(self.proc, self.basis, c)
            if np.linalg.matrix_rank(b, tol=1e-9 * np.abs(b).max()) == self.rank:
                break
            m *= 2
        cd = np.stack([diagram_colour_values(t, rk, self.proc, c) for t, rk in self.diagrams], axis=1)
        coef, *_ = np.linalg.lstsq(b, cd, rcond=1e-10)
        self.coef = coef.T.copy()                                # [D, K]
        # independent check on fresh assignments
        cv = random_assignments(self.proc, 512, seed + 1)
        bv = basis_values(self.proc, self.basis, cv)
        dv = np.stack([diagram_colour_values(t, rk, self.proc, cv) for t, rk in self.diagrams], axis=1)
        self.decomposition_residual = float(np.max(np.abs(bv @ coef - dv))) if d else 0.0
        assert self.decomposition_residual < 1e-9, self.decomposition_residual

    def distinct_nonzero(self) -> int:
        """Distinct non-zero values on and above the diagonal of N (Table 3)."""
        k = len(self.basis)
        vals = {self.N_frac[i][j] for i in range(k) for j in range(i, k)}
        vals.discard(Fraction(0))
        return len(vals)


@functools.lru_cache(maxsize=None)
def colour_data(spec: str) -> ColourData:
    return ColourData(parse_process(spec).spec)
