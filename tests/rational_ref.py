"""Exact rational re-execution of the set-up and the preconditioned RCG.

Every step of Alg. 2 (Sec. 3.2) and Alg. 3 (Sec. 3.4.1) on a fixed pattern
is rational in its inputs: the local min-norm correction is
G_i (G_i^T G_i)^{-1} r_i, the row projector is I - G_i (G_i^T G_i)^{-1} G_i^T,
the masked product and the (block) Jacobi scaling are sums, products and
small linear solves, and the CG scalars are quotients of inner products.
On inputs made of small integers the whole path can therefore be run in
exact arithmetic with ``fractions.Fraction``, which gives the exact k-th
iterate against which the FP64 oracle is held.

This route shares nothing with the oracle: no QR or SVD (the Gram matrix is
solved by exact Gauss-Jordan elimination), no scipy, dictionaries instead of
CSR arrays, and the projector applied through the Gram matrix rather than an
orthonormal basis.  Only rows with full-rank G_i are handled (the exact rank
is checked; the SVD branch of Alg. 2 has its own pins).
"""

from fractions import Fraction


class RankDeficient(Exception):
    pass


def _solve(M, b):
    """Exact solution of the square system M x = b (lists of Fractions) by
    Gauss-Jordan elimination with a non-zero pivot; raises RankDeficient when
    M is singular."""
    n = len(M)
    aug = [list(M[i]) + [b[i]] for i in range(n)]
    for c in range(n):
        piv = next((r for r in range(c, n) if aug[r][c] != 0), None)
        if piv is None:
            raise RankDeficient
        aug[c], aug[piv] = aug[piv], aug[c]
        p = aug[c][c]
        aug[c] = [v / p for v in aug[c]]
        for r in range(n):
            if r != c and aug[r][c] != 0:
                f = aug[r][c]
                aug[r] = [vr - f * vc for vr, vc in zip(aug[r], aug[c])]
    return [aug[i][n] for i in range(n)]


class ExactProblem:
    """A (dict of dicts), the pattern rows J_i, P0 on the pattern, B, B_c,
    all as Fractions."""

    def __init__(self, A, P0, B, Bc, rowptr, colind):
        A = A.tocsr()
        self.n = A.shape[0]
        self.m = Bc.shape[1]
        self.A = [dict() for _ in range(self.n)]
        for i in range(self.n):
            for t in range(A.indptr[i], A.indptr[i + 1]):
                self.A[i][int(A.indices[t])] = Fraction(float(A.data[t]))
        P0 = P0.tocsr()
        p0 = [dict() for _ in range(self.n)]
        for i in range(self.n):
            for t in range(P0.indptr[i], P0.indptr[i + 1]):
                p0[i][int(P0.indices[t])] = Fraction(float(P0.data[t]))
        self.J = [[int(c) for c in colind[rowptr[i]:rowptr[i + 1]]] for i in range(self.n)]
        self.B = [[Fraction(float(v)) for v in row] for row in B]
        self.Bc = [[Fraction(float(v)) for v in row] for row in Bc]
        # P0 placed on the pattern (every P0 entry lies in it)
        self.p_hat = [[p0[i].get(j, Fraction(0)) for j in self.J[i]] for i in range(self.n)]
        assert all(set(p0[i]) <= set(self.J[i]) for i in range(self.n))

    # ---- Alg. 2 through the Gram matrix ---------------------------------
    def gram(self, i):
        G = [self.Bc[j] for j in self.J[i]]
        return G, [[sum(G[s][a] * G[s][b] for s in range(len(G))) for b in range(self.m)]
                   for a in range(self.m)]

    def setup(self):
        """p0'_i = p_hat_i + G_i (G_i^T G_i)^{-1} (b_i - G_i^T p_hat_i)."""
        out = []
        for i in range(self.n):
            G, M = self.gram(i)
            r = [self.B[i][c] - sum(G[s][c] * self.p_hat[i][s] for s in range(len(G)))
                 for c in range(self.m)]
            w = _solve(M, r)
            out.append([self.p_hat[i][s] + sum(G[s][c] * w[c] for c in range(self.m))
                        for s in range(len(G))])
        return out

    def project(self, X):
        """Pi_i x = x - G_i (G_i^T G_i)^{-1} G_i^T x, row by row."""
        out = []
        for i in range(self.n):
            G, M = self.gram(i)
            g = [sum(G[s][c] * X[i][s] for s in range(len(G))) for c in range(self.m)]
            w = _solve(M, g)
            out.append([X[i][s] - sum(G[s][c] * w[c] for c in range(self.m))
                        for s in range(len(G))])
        return out

    # ---- K y: (A Y)(i, j) for j in J_i --------------------------------------
    def masked_product(self, X):
        out = []
        for i in range(self.n):
            acc = {j: Fraction(0) for j in self.J[i]}
            for k, a in self.A[i].items():
                for s, j in enumerate(self.J[k]):
                    if j in acc:
                        acc[j] += a * X[k][s]
            out.append([acc[j] for j in self.J[i]])
        return out

    # ---- preconditioners --------------------------------------------------
    def jacobi(self, X):
        return [[v / self.A[i][i] for v in X[i]] for i in range(self.n)]

    def block_jacobi(self, X, bs):
        """For node a (rows bs*a .. bs*a + bs - 1) and column j, solve with
        the sub-block of A on the node's rows whose pattern holds j."""
        out = [[None] * len(self.J[i]) for i in range(self.n)]
        for a in range(self.n // bs):
            rows = list(range(bs * a, bs * a + bs))
            cols = sorted({j for i in rows for j in self.J[i]})
            for j in cols:
                sub = [i for i in rows if j in self.J[i]]
                pos = [self.J[i].index(j) for i in sub]
                M = [[self.A[i].get(k, Fraction(0)) for k in sub] for i in sub]
                z = _solve(M, [X[i][p] for i, p in zip(sub, pos)])
                for i, p, v in zip(sub, pos, z):
                    out[i][p] = v
        return out

    @staticmethod
    def dot(X, Y):
        return sum(x * y for rx, ry in zip(X, Y) for x, y in zip(rx, ry))

    @staticmethod
    def axpy(alpha, X, Y):
        return [[alpha * x + y for x, y in zip(rx, ry)] for rx, ry in zip(X, Y)]

    def energy(self, P):
        return self.dot(P, self.masked_product(P))

    def rcg(self, iters, precond="jacobi", bs=1):
        """The exact iterate after ``iters`` steps of the projected PCG with
        the Pi M^{-1} Pi preconditioner, started from the corrected P0.
        Returns (P, [E(P_0), ..., E(P_iters)])."""
        w0 = self.setup()
        r = [[-v for v in row] for row in self.project(self.masked_product(w0))]
        dw = [[Fraction(0)] * len(row) for row in w0]
        energies = [self.energy(w0)]
        y, gamma_prev = None, None
        for k in range(iters):
            z = self.jacobi(r) if precond == "jacobi" else self.block_jacobi(r, bs)
            z = self.project(z)
            gamma = self.dot(r, z)
            assert gamma > 0
            y = z if k == 0 else self.axpy(gamma / gamma_prev, y, z)
            gamma_prev = gamma
            yh = self.project(self.masked_product(y))
            d = self.dot(y, yh)
            assert d > 0
            alpha = gamma / d
            dw = self.axpy(alpha, y, dw)
            r = self.axpy(-alpha, yh, r)
            energies.append(self.energy(self.axpy(Fraction(1), dw, w0)))
        return self.axpy(Fraction(1), dw, w0), energies


def flatten(X):
    return [float(v) for row in X for v in row]
