"""Exact complex-rational arithmetic for pinning the oracle on tiny inputs.

Independent of the oracle: it implements Gaussian-rational numbers, exact
Gauss-Jordan elimination and the Krylov-subspace characterisation of CG
iterates, none of which the oracle uses.
"""

from fractions import Fraction


class QC:
    """Complex number with exact rational real and imaginary parts."""

    __slots__ = ("re", "im")

    def __init__(self, re=0, im=0):
        self.re = Fraction(re)
        self.im = Fraction(im)

    def __add__(self, o):
        o = _q(o)
        return QC(self.re + o.re, self.im + o.im)

    __radd__ = __add__

    def __sub__(self, o):
        o = _q(o)
        return QC(self.re - o.re, self.im - o.im)

    def __rsub__(self, o):
        return _q(o) - self

    def __neg__(self):
        return QC(-self.re, -self.im)

    def __mul__(self, o):
        o = _q(o)
        return QC(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    __rmul__ = __mul__

    def conj(self):
        return QC(self.re, -self.im)

    def abs2(self):
        return self.re * self.re + self.im * self.im

    def __truediv__(self, o):
        o = _q(o)
        den = o.abs2()
        n = self * o.conj()
        return QC(n.re / den, n.im / den)

    def __eq__(self, o):
        o = _q(o)
        return self.re == o.re and self.im == o.im

    def __complex__(self):
        return complex(float(self.re), float(self.im))

    def __repr__(self):
        return f"QC({self.re}, {self.im})"


def _q(x):
    if isinstance(x, QC):
        return x
    if isinstance(x, complex):
        return QC(Fraction(x.real), Fraction(x.imag))
    return QC(x, 0)


def mat(rows):
    return [[_q(v) for v in r] for r in rows]


def matmul(A, B):
    n, k, m = len(A), len(B), len(B[0])
    return [[sum((A[i][t] * B[t][j] for t in range(k)), QC()) for j in range(m)] for i in range(n)]


def adjoint(A):
    return [[A[j][i].conj() for j in range(len(A))] for i in range(len(A[0]))]


def identity(n):
    return [[QC(1 if i == j else 0) for j in range(n)] for i in range(n)]


def solve(A, B):
    """Exact solution of A X = B by Gauss-Jordan elimination (any nonsingular A)."""
    n = len(A)
    m = len(B[0])
    aug = [list(A[i]) + list(B[i]) for i in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if not aug[r][c] == QC())
        aug[c], aug[p] = aug[p], aug[c]
        piv = aug[c][c]
        aug[c] = [v / piv for v in aug[c]]
        for r in range(n):
            if r != c and not aug[r][c] == QC():
                f = aug[r][c]
                aug[r] = [a - f * b for a, b in zip(aug[r], aug[c])]
    return [row[n:] for row in aug]


def krylov_optimal_iterate(A, b, t, dinv):
    """x_t = argmin over span{z0, N z0, ..., N^{t-1} z0} of the A-norm error,
    with N = D^{-1} A and z0 = D^{-1} b.

    For any basis V of that subspace, x_t = V (V^H A V)^{-1} V^H b. This is the
    defining optimality of the t-th preconditioned CG iterate (started at 0),
    stated without any of the CG recurrences.
    """
    K = len(A)
    z = [[dinv[i] * b[i][0]] for i in range(K)]
    cols = [z]
    for _ in range(t - 1):
        Az = matmul(A, cols[-1])
        cols.append([[dinv[i] * Az[i][0]] for i in range(K)])
    V = [[cols[c][i][0] for c in range(t)] for i in range(K)]
    VH = adjoint(V)
    G = matmul(VH, matmul(A, V))
    rhs = matmul(VH, b)
    y = solve(G, rhs)
    return matmul(V, y)
