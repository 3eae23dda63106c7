"""Particle/grid weights of Sec. 3.1 (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A point X in the periodic box with grid spacing h = L/H has cell index
g = floor(X/h) and relative position lambda = X/h - g in [0,1)^3
(Sec. 3.1, below eq. ``2ord``).  A stencil is a list of integer offsets gamma
and weights F_gamma(lambda); node g + gamma is stored at (g + gamma) mod H.

* Order 2, Gamma_2 = {0,1}^3, F^(2)_j = prod_s (1 - j_s + (2 j_s - 1) lambda_s)
  (eq. ``2ord``): trilinear weights.
* Order 4, Gamma_4 = Gamma_2 plus the 24 "outer" nodes that have exactly one
  coordinate in {-1, 2} and the other two in {0,1} (Sec. 3.1).  Eq. ``4ord``
  prints the inner weights and the two outer rows along axis 1, and elides the
  remaining rows with dots while stating that the weights have cubic symmetry.
  Reading taken: the axis-2 and axis-3 outer rows are the axis-1 rows with the
  axes permuted, i.e. for an outer node on axis a
      F_{..2..}  = -(1 + l_a)(1 - l_a) l_a / 6 * prod_{s != a} w_{j_s}(l_s)
      F_{..-1..} = -(2 - l_a) l_a (1 - l_a) / 6 * prod_{s != a} w_{j_s}(l_s)
  with w_0(l) = 1 - l, w_1(l) = l; the inner weights are
      F_j = prod_s w_{j_s}(l_s) * (1 + sum_k l_k (1 - l_k) / 2).

Two dimensions (the 2-D experiments of Sec. 5.2 use "fourth-order
particle-to-grid" without printing the weights).  Reading taken: the same
construction with d = 2, Gamma_4 = {0,1}^2 plus the 8 nodes with one
coordinate in {-1, 2} and the other in {0,1}; the inner correction sums over
the two axes.  The weights still sum to one and reproduce polynomials of
degree 3 (pinned).
"""

import itertools

import numpy as np

# 32 offsets of Gamma_4: the 8 inner nodes, then for each axis a the outer nodes
# (-1 then 2 on axis a) crossed with {0,1}^2 on the other two axes.
_INNER = [tuple(j) for j in itertools.product((0, 1), repeat=3)]
_OUTER = []
for _a in range(3):
    for _e in (-1, 2):
        for _j in itertools.product((0, 1), repeat=2):
            _o = list(_j)
            _o.insert(_a, _e)
            _OUTER.append((tuple(_o), _a))

OFFSETS2 = np.array(_INNER, dtype=np.int64)                       # (8, 3)
OFFSETS4 = np.array(_INNER + [o for o, _ in _OUTER], dtype=np.int64)  # (32, 3)


def _w(j, lam):
    """Linear hat factor w_j(l): 1 - l for j = 0, l for j = 1."""
    return 1.0 - lam if j == 0 else lam


def _dw(j):
    return -1.0 if j == 0 else 1.0


def _outer1d(e, lam):
    """One-axis factor of an outer node: e = 2 or e = -1 (eq. 4ord)."""
    if e == 2:
        return -(1.0 + lam) * (1.0 - lam) * lam / 6.0
    return -(2.0 - lam) * lam * (1.0 - lam) / 6.0


def _douter1d(e, lam):
    """d/dl of ``_outer1d``: -(l - l^3)/6 and -(2l - 3l^2 + l^3)/6."""
    if e == 2:
        return -(1.0 - 3.0 * lam * lam) / 6.0
    return -(2.0 - 6.0 * lam + 3.0 * lam * lam) / 6.0


def offsets(order):
    return OFFSETS2 if order == 2 else OFFSETS4


def weights(lam, order):
    """F_gamma(lambda) for every offset; lam (..., 3) -> (..., n_nodes)."""
    lam = np.asarray(lam, dtype=np.float64)
    l1, l2, l3 = lam[..., 0], lam[..., 1], lam[..., 2]
    ls = (l1, l2, l3)
    cols = []
    if order == 2:
        for j in _INNER:
            cols.append(_w(j[0], l1) * _w(j[1], l2) * _w(j[2], l3))
        return np.stack(cols, axis=-1)
    if order != 4:
        raise ValueError("order must be 2 or 4")
    S = 1.0 + (l1 * (1.0 - l1) + l2 * (1.0 - l2) + l3 * (1.0 - l3)) / 2.0
    for j in _INNER:
        cols.append(_w(j[0], l1) * _w(j[1], l2) * _w(j[2], l3) * S)
    for o, a in _OUTER:
        f = _outer1d(o[a], ls[a])
        for s in range(3):
            if s != a:
                f = f * _w(o[s], ls[s])
        cols.append(f)
    return np.stack(cols, axis=-1)


def dweights(lam, order):
    """d F_gamma / d lambda_a; lam (..., 3) -> (..., n_nodes, 3)."""
    lam = np.asarray(lam, dtype=np.float64)
    ls = (lam[..., 0], lam[..., 1], lam[..., 2])
    out = []
    if order == 2:
        for j in _INNER:
            d = []
            for a in range(3):
                f = _dw(j[a]) * np.ones_like(ls[a])
                for s in range(3):
                    if s != a:
                        f = f * _w(j[s], ls[s])
                d.append(f)
            out.append(np.stack(d, axis=-1))
        return np.stack(out, axis=-2)
    S = 1.0 + sum(l * (1.0 - l) for l in ls) / 2.0
    for j in _INNER:
        W = _w(j[0], ls[0]) * _w(j[1], ls[1]) * _w(j[2], ls[2])
        d = []
        for a in range(3):
            dW = _dw(j[a]) * np.ones_like(ls[a])
            for s in range(3):
                if s != a:
                    dW = dW * _w(j[s], ls[s])
            d.append(dW * S + W * (1.0 - 2.0 * ls[a]) / 2.0)
        out.append(np.stack(d, axis=-1))
    for o, a in _OUTER:
        d = []
        for b in range(3):
            if b == a:
                f = _douter1d(o[a], ls[a])
            else:
                f = _outer1d(o[a], ls[a]) * _dw(o[b])
            for s in range(3):
                if s != a and s != b:
                    f = f * _w(o[s], ls[s])
            d.append(f)
        out.append(np.stack(d, axis=-1))
    return np.stack(out, axis=-2)


# ---------------------------------------------------------------------------
# two dimensions
# ---------------------------------------------------------------------------
_INNER2 = [tuple(j) for j in itertools.product((0, 1), repeat=2)]
_OUTER2 = []
for _a in range(2):
    for _e in (-1, 2):
        for _j in (0, 1):
            _o = [_j]
            _o.insert(_a, _e)
            _OUTER2.append((tuple(_o), _a))

OFFSETS2_2D = np.array(_INNER2, dtype=np.int64)                           # (4, 2)
OFFSETS4_2D = np.array(_INNER2 + [o for o, _ in _OUTER2], dtype=np.int64)  # (12, 2)


def offsets2d(order):
    return OFFSETS2_2D if order == 2 else OFFSETS4_2D


def weights2d(lam, order):
    """F_gamma(lambda) in two dimensions; lam (..., 2) -> (..., n_nodes)."""
    lam = np.asarray(lam, dtype=np.float64)
    ls = (lam[..., 0], lam[..., 1])
    cols = []
    if order == 2:
        for j in _INNER2:
            cols.append(_w(j[0], ls[0]) * _w(j[1], ls[1]))
        return np.stack(cols, axis=-1)
    if order != 4:
        raise ValueError("order must be 2 or 4")
    S = 1.0 + (ls[0] * (1.0 - ls[0]) + ls[1] * (1.0 - ls[1])) / 2.0
    for j in _INNER2:
        cols.append(_w(j[0], ls[0]) * _w(j[1], ls[1]) * S)
    for o, a in _OUTER2:
        b = 1 - a
        cols.append(_outer1d(o[a], ls[a]) * _w(o[b], ls[b]))
    return np.stack(cols, axis=-1)
