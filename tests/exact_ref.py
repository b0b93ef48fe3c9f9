"""Exact-rational statement of the wavelet stage, for pinning the oracle.

Independent of the oracle's derivation: predictions come from fitting the
polynomial itself (a Vandermonde solve over Fractions) rather than from
Lagrange weight formulas, the W4_li update from the transposed predict matrix,
and the W3_ai prediction from integrating the fitted quadratic.  Paper sections
named are those of arXiv 1903.07761 (Sec. 2.3, "Wavelet-based compression" and
"Wavelet types"); the stencil readings are the ones stated in the oracle's
header.  Pure Python, meant for small inputs only.
"""
from __future__ import annotations

from fractions import Fraction as F
from functools import lru_cache

W4, W4LI, W3AI = 0, 1, 2


def _solve(A, b):
    """Gaussian elimination over Fractions (A square, nonsingular)."""
    n = len(A)
    M = [list(map(F, row)) + [F(v)] for row, v in zip(A, b)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [a - f * bb for a, bb in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


def nearest(count, avail, pos):
    """The `count` available integer sites nearest to pos (ascending)."""
    order = sorted(range(avail), key=lambda k: (abs(F(k) - pos), k))
    return sorted(order[:count])


def poly_fit_eval(xs, ys, t):
    """Value at t of the polynomial of degree len(xs)-1 through (xs, ys)."""
    n = len(xs)
    coef = _solve([[F(x) ** p for p in range(n)] for x in xs], ys)
    return sum(c * F(t) ** p for p, c in enumerate(coef))


@lru_cache(maxsize=None)
def w4_predict_row(h, m):
    """Row m of the W4 predict matrix: weights over evens 0..h-1, obtained by
    fitting the cubic through the four nearest existing evens to unit data."""
    nodes = nearest(4, h, F(2 * m + 1, 2))
    row = [F(0)] * h
    for k in nodes:
        ys = [F(1) if j == k else F(0) for j in nodes]
        row[k] = poly_fit_eval(nodes, ys, F(2 * m + 1, 2))
    return tuple(row)


@lru_cache(maxsize=None)
def w4li_update_col(h, m):
    """Column m of the W4_li update U = P~^T / 2 over evens 0..h-1: P~ row m is
    the cubic fitted through the centred evens m-1..m+2 (wherever they lie),
    evaluated at m + 1/2; only the weights on existing evens are used."""
    nodes = [m - 1, m, m + 1, m + 2]
    col = [F(0)] * h
    for k in nodes:
        if 0 <= k < h:
            ys = [F(1) if j == k else F(0) for j in nodes]
            col[k] = poly_fit_eval(nodes, ys, F(2 * m + 1, 2)) / 2
    return tuple(col)


def w3_predict(C, k):
    """Average over [k, k+1/2] of the quadratic whose averages over the three
    nearest existing coarse cells equal C there (cell j = [j, j+1])."""
    h = len(C)
    cells = nearest(3, h, F(k))  # by distance between cell centres
    # unknown quadratic a + b x + c x^2; its average over [j, j+1]:
    rows = [[F(1), F(2 * j + 1, 2), (F(j + 1) ** 3 - F(j) ** 3) / 3] for j in cells]
    a, b, c = _solve(rows, [C[j] for j in cells])
    lo, hi = F(k), F(k) + F(1, 2)
    integral = a * (hi - lo) + b * (hi ** 2 - lo ** 2) / 2 + c * (hi ** 3 - lo ** 3) / 3
    return integral * 2


def fwd1(scheme, v):
    n = len(v)
    h = n // 2
    v = [F(x) for x in v]
    if scheme == W3AI:
        C = [(v[2 * k] + v[2 * k + 1]) / 2 for k in range(h)]
        d = [v[2 * k] - w3_predict(C, k) for k in range(h)]
        return C + d
    e = v[0::2]
    o = v[1::2]
    P = [w4_predict_row(h, m) for m in range(h)]
    d = [o[m] - sum(P[m][k] * e[k] for k in range(h)) for m in range(h)]
    if scheme == W4LI:
        e = [e[k] + sum(w4li_update_col(h, m)[k] * d[m] for m in range(h)) for k in range(h)]
    return e + d


def inv1(scheme, w):
    n = len(w)
    h = n // 2
    w = [F(x) for x in w]
    s, d = w[:h], w[h:]
    v = [F(0)] * n
    if scheme == W3AI:
        for k in range(h):
            a = w3_predict(s, k) + d[k]
            v[2 * k] = a
            v[2 * k + 1] = 2 * s[k] - a
        return v
    P = [w4_predict_row(h, m) for m in range(h)]
    e = list(s)
    if scheme == W4LI:
        e = [s[k] - sum(w4li_update_col(h, m)[k] * d[m] for m in range(h)) for k in range(h)]
    for k in range(h):
        v[2 * k] = e[k]
    for m in range(h):
        v[2 * m + 1] = d[m] + sum(P[m][k] * e[k] for k in range(h))
    return v


def fwd_line(scheme, v):
    v = [F(x) for x in v]
    n = len(v)
    while n >= 8:
        v[:n] = fwd1(scheme, v[:n])
        n //= 2
    return v


def _axis_lines(N, n, axis):
    """Index lists (q = x + N(y + N z)) of every line along axis in [0,n)^3."""
    for a in range(n):
        for b in range(n):
            if axis == 0:
                yield [x + N * (a + N * b) for x in range(n)]
            elif axis == 1:
                yield [a + N * (y + N * b) for y in range(n)]
            else:
                yield [a + N * (b + N * z) for z in range(n)]


def fwd_block(scheme, B, N):
    """B: flat list of N^3 values (q = x + N(y + N z)); exact forward."""
    B = [F(x) for x in B]
    n = N
    while n >= 8:
        for axis in (0, 1, 2):
            for idx in _axis_lines(N, n, axis):
                out = fwd1(scheme, [B[i] for i in idx])
                for i, val in zip(idx, out):
                    B[i] = val
        n //= 2
    return B


def inv_block(scheme, C, N):
    C = [F(x) for x in C]
    n = 8
    while n <= N:
        for axis in (2, 1, 0):
            for idx in _axis_lines(N, n, axis):
                out = inv1(scheme, [C[i] for i in idx])
                for i, val in zip(idx, out):
                    C[i] = val
        n *= 2
    return C


# ---------------------------------------------------------------------------
# Rounded replay: the same readings with every operation rounded in a given
# precision, in the documented order (weighted sums left to right in ascending
# source index, starting from the first term; no fused multiply-add).  The
# weights are the exact rationals above, which every precision holds exactly.
# numpy scalar arithmetic rounds each operation to its dtype.

def _dot(ws, xs, dt):
    acc = dt(ws[0]) * xs[0]
    for w, x in zip(ws[1:], xs[1:]):
        acc = acc + dt(w) * x
    return acc


@lru_cache(maxsize=None)
def _w3_weights(h, k):
    """W3_ai predict weights over its three cells (from w3_predict on units)."""
    cells = nearest(3, h, F(k))
    ws = []
    for j in cells:
        unit = [F(1) if i == j else F(0) for i in range(h)]
        ws.append(w3_predict(unit, k))
    return tuple(cells), tuple(ws)


def rounded_fwd1(scheme, v, dt):
    n = len(v)
    h = n // 2
    v = [dt(x) for x in v]
    if scheme == W3AI:
        C = [(v[2 * k] + v[2 * k + 1]) * dt(0.5) for k in range(h)]
        d = []
        for k in range(h):
            cells, ws = _w3_weights(h, k)
            d.append(v[2 * k] - _dot([float(w) for w in ws], [C[j] for j in cells], dt))
        return C + d
    e, o = v[0::2], v[1::2]
    d = []
    for m in range(h):
        row = w4_predict_row(h, m)
        ks = [k for k in range(h) if row[k] != 0]
        d.append(o[m] - _dot([float(row[k]) for k in ks], [e[k] for k in ks], dt))
    if scheme == W4LI:
        s = []
        for k in range(h):
            terms = [(float(w4li_update_col(h, m)[k]), d[m]) for m in range(h) if w4li_update_col(h, m)[k] != 0]
            s.append(e[k] + _dot([t[0] for t in terms], [t[1] for t in terms], dt))
        e = s
    return e + d


def rounded_fwd_block(scheme, B, N, dt):
    B = [dt(x) for x in B]
    n = N
    while n >= 8:
        for axis in (0, 1, 2):
            for idx in _axis_lines(N, n, axis):
                out = rounded_fwd1(scheme, [B[i] for i in idx], dt)
                for i, val in zip(idx, out):
                    B[i] = val
        n //= 2
    return B


def rounded_inv1(scheme, w, dt):
    n = len(w)
    h = n // 2
    w = [dt(x) for x in w]
    s, d = w[:h], w[h:]
    v = [dt(0)] * n
    if scheme == W3AI:
        for k in range(h):
            cells, ws = _w3_weights(h, k)
            a = _dot([float(x) for x in ws], [s[j] for j in cells], dt) + d[k]
            v[2 * k] = a
            v[2 * k + 1] = (s[k] + s[k]) - a
        return v
    e = list(s)
    if scheme == W4LI:
        e = []
        for k in range(h):
            terms = [(float(w4li_update_col(h, m)[k]), d[m]) for m in range(h) if w4li_update_col(h, m)[k] != 0]
            e.append(s[k] - _dot([t[0] for t in terms], [t[1] for t in terms], dt))
    for k in range(h):
        v[2 * k] = e[k]
    for m in range(h):
        row = w4_predict_row(h, m)
        ks = [k for k in range(h) if row[k] != 0]
        v[2 * m + 1] = d[m] + _dot([float(row[k]) for k in ks], [e[k] for k in ks], dt)
    return v


def rounded_inv_block(scheme, C, N, dt):
    C = [dt(x) for x in C]
    n = 8
    while n <= N:
        for axis in (2, 1, 0):
            for idx in _axis_lines(N, n, axis):
                out = rounded_inv1(scheme, [C[i] for i in idx], dt)
                for i, val in zip(idx, out):
                    C[i] = val
        n *= 2
    return C
