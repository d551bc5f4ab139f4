"""Exact reference data for pinning the oracle (test infrastructure).

Everything here is evaluated from textbook ADM general relativity, not from
the Z4c equations the oracle implements:

* the ADM (York) evolution equations with matter,
      d_t gamma_ij = -2 alpha K_ij + L_beta gamma_ij
      d_t K_ij     = -D_i D_j alpha + alpha (R_ij - 2 K_ik K^k_j + K K_ij)
                     - 8 pi alpha (S_ij - gamma_ij (S - rho) / 2) + L_beta K_ij
* the ADM constraints, used to *define* matter that satisfies them,
      16 pi rho = R + K^2 - K_ij K^ij,    8 pi S_i = D_j K^j_i - D_i K,
* the Ricci tensor from Christoffel symbols,
      R_ij = d_k G^k_ij - d_j G^k_ik + G^k_kl G^l_ij - G^k_jl G^l_ik,
* the change of variables ADM -> Z4c (chi = det(gamma)^(-1/3),
  gt = chi gamma, Khat = K with Theta = 0, At = chi (K_ij - gamma_ij K / 3),
  Gt^i = gt^{jk} Gt^i_jk) and its time derivative by the chain rule.

Derivatives are exact (to rounding): every quantity is a second-order Taylor
jet in (x, y, z) propagated by forward-mode differentiation (Leibniz and
chain rules), so no finite differences enter the reference values.

Exact spacetimes provided: Kerr-Schild Schwarzschild (static, shifted), the
1-D and the diagonal gauge waves (harmonic slicing, an exact solution whose
fields depend on x - t only), and generic smooth ADM data with matter chosen
to satisfy the constraints.
"""
from __future__ import annotations

import math

import numpy as np

SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
FIELDS = ["chi", "gxx", "gxy", "gxz", "gyy", "gyz", "gzz", "Khat",
          "Axx", "Axy", "Axz", "Ayy", "Ayz", "Azz", "Theta",
          "Gx", "Gy", "Gz", "alpha", "bx", "by", "bz"]


class Jet:
    """Value with its first and second partial derivatives in (x, y, z),
    truncated at `order` (2, 1 or 0).  Arithmetic propagates derivatives."""
    __slots__ = ("v", "d", "dd", "order")

    def __init__(self, v, d=None, dd=None, order=2):
        self.v = v
        self.order = order
        self.d = d if order >= 1 else None
        self.dd = dd if order >= 2 else None

    @staticmethod
    def const(c, shape):
        z = np.zeros(shape)
        return Jet(np.full(shape, float(c)), [z] * 3, [[z] * 3 for _ in range(3)], 2)

    @staticmethod
    def coord(k, X):
        z = np.zeros_like(X)
        o = np.ones_like(X)
        return Jet(X.copy(), [o if a == k else z for a in range(3)],
                   [[z] * 3 for _ in range(3)], 2)

    def _lift(self, other):
        if isinstance(other, Jet):
            return other
        return Jet.const(other, np.shape(self.v))

    def __add__(self, o):
        o = self._lift(o)
        n = min(self.order, o.order)
        d = [self.d[i] + o.d[i] for i in range(3)] if n >= 1 else None
        dd = [[self.dd[i][j] + o.dd[i][j] for j in range(3)] for i in range(3)] if n >= 2 else None
        return Jet(self.v + o.v, d, dd, n)

    __radd__ = __add__

    def __neg__(self):
        d = [-a for a in self.d] if self.order >= 1 else None
        dd = [[-a for a in r] for r in self.dd] if self.order >= 2 else None
        return Jet(-self.v, d, dd, self.order)

    def __sub__(self, o):
        return self + (-self._lift(o))

    def __rsub__(self, o):
        return self._lift(o) + (-self)

    def __mul__(self, o):
        if not isinstance(o, Jet):
            c = float(o)
            d = [c * a for a in self.d] if self.order >= 1 else None
            dd = [[c * a for a in r] for r in self.dd] if self.order >= 2 else None
            return Jet(c * self.v, d, dd, self.order)
        n = min(self.order, o.order)
        d = dd = None
        if n >= 1:
            d = [self.d[i] * o.v + self.v * o.d[i] for i in range(3)]
        if n >= 2:
            dd = [[self.dd[i][j] * o.v + self.d[i] * o.d[j] + self.d[j] * o.d[i]
                   + self.v * o.dd[i][j] for j in range(3)] for i in range(3)]
        return Jet(self.v * o.v, d, dd, n)

    __rmul__ = __mul__

    def apply(self, f0, f1, f2):
        """Chain rule for a scalar function with derivatives f1 = f', f2 = f''."""
        v = f0(self.v)
        d = dd = None
        if self.order >= 1:
            a1 = f1(self.v)
            d = [a1 * self.d[i] for i in range(3)]
        if self.order >= 2:
            a2 = f2(self.v)
            dd = [[a2 * self.d[i] * self.d[j] + a1 * self.dd[i][j] for j in range(3)]
                  for i in range(3)]
        return Jet(v, d, dd, self.order)

    def recip(self):
        return self.apply(lambda u: 1.0 / u, lambda u: -1.0 / (u * u),
                          lambda u: 2.0 / (u * u * u))

    def __truediv__(self, o):
        if not isinstance(o, Jet):
            return self * (1.0 / float(o))
        return self * o.recip()

    def __rtruediv__(self, o):
        return self.recip() * float(o)

    def __pow__(self, p):
        p = float(p)
        return self.apply(lambda u: u ** p, lambda u: p * u ** (p - 1.0),
                          lambda u: p * (p - 1.0) * u ** (p - 2.0))

    def diff(self, k):
        """d/dx_k: a jet of one order less."""
        assert self.order >= 1
        n = self.order - 1
        d = [self.dd[k][i] for i in range(3)] if n >= 1 else None
        return Jet(self.d[k], d, None, n)


def jsin(a):
    return a.apply(np.sin, np.cos, lambda u: -np.sin(u))


def jcos(a):
    return a.apply(np.cos, lambda u: -np.sin(u), lambda u: -np.cos(u))


def jsqrt(a):
    return a ** 0.5


def det3(g):
    return (g[0][0] * (g[1][1] * g[2][2] - g[1][2] * g[2][1])
            - g[0][1] * (g[1][0] * g[2][2] - g[1][2] * g[2][0])
            + g[0][2] * (g[1][0] * g[2][1] - g[1][1] * g[2][0]))


def inv3(g):
    d = det3(g)
    rd = d.recip()
    adj = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            # cofactor C_ji -> (i, j) entry of the inverse
            r = [a for a in range(3) if a != j]
            c = [b for b in range(3) if b != i]
            m = g[r[0]][c[0]] * g[r[1]][c[1]] - g[r[0]][c[1]] * g[r[1]][c[0]]
            adj[i][j] = m * rd if (i + j) % 2 == 0 else -(m * rd)
    return adj


def christoffel(g, gi):
    dg = [[[g[i][j].diff(k) for j in range(3)] for i in range(3)] for k in range(3)]
    low = [[[(dg[i][j][k] + dg[j][i][k] - dg[k][i][j]) * 0.5 for j in range(3)]
            for i in range(3)] for k in range(3)]
    up = [[[sum((gi[k][l] * low[l][i][j] for l in range(1, 3)), gi[k][0] * low[0][i][j])
            for j in range(3)] for i in range(3)] for k in range(3)]
    return low, up


def _sum(it):
    it = list(it)
    s = it[0]
    for a in it[1:]:
        s = s + a
    return s


def lie_sym(T, beta):
    return [[_sum(beta[k] * T[i][j].diff(k) + T[i][k] * beta[k].diff(j)
                  + T[k][j] * beta[k].diff(i) for k in range(3)) for j in range(3)]
            for i in range(3)]


def ricci(G):
    R = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            R[i][j] = (_sum(G[k][i][j].diff(k) for k in range(3))
                       - _sum(G[k][i][k].diff(j) for k in range(3))
                       + _sum(G[k][k][l] * G[l][i][j] - G[k][j][l] * G[l][i][k]
                              for k in range(3) for l in range(3)))
    return R


def matmul(A, B):
    return [[_sum(A[i][k] * B[k][j] for k in range(3)) for j in range(3)] for i in range(3)]


def trace_with(gi, T):
    return _sum(gi[i][j] * T[i][j] for i in range(3) for j in range(3))


def z4c_from_adm(g, K, alpha, beta):
    """Z4c variables (values only) of ADM data given as jets."""
    gi = inv3(g)
    trK = trace_with(gi, K)
    chi = det3(g) ** (-1.0 / 3.0)
    gt = [[chi * g[i][j] for j in range(3)] for i in range(3)]
    git = [[gi[i][j] / chi for j in range(3)] for i in range(3)]
    _, up = christoffel(gt, git)
    out = {"chi": chi.v, "Khat": trK.v, "Theta": np.zeros_like(chi.v), "alpha": alpha.v}
    for a, (i, j) in enumerate(SYM):
        out[FIELDS[1 + a]] = gt[i][j].v
        out[FIELDS[8 + a]] = (chi * (K[i][j] - g[i][j] * trK * (1.0 / 3.0))).v
    for i in range(3):
        out[FIELDS[15 + i]] = trace_with(git, [[up[i][j][k] for k in range(3)]
                                               for j in range(3)]).v
    for i in range(3):
        out[FIELDS[19 + i]] = beta[i].v
    return out


def adm_evolution(g, K, alpha, beta, Sij=None, constraint_matter=False):
    """Returns (dt of the Z4c variables with frozen gauge, matter list of 10
    arrays rho, S_i, S_ij).  With constraint_matter, rho and S_i are defined
    by the ADM constraints so that H = M_i = 0 hold exactly."""
    shape = np.shape(g[0][0].v)
    zero = Jet.const(0.0, shape)
    gi = inv3(g)
    _, G = christoffel(g, gi)
    R = ricci(G)
    trK = trace_with(gi, K)
    Kmix = matmul(gi, K)                    # K^i_j
    KK = _sum(Kmix[i][j] * Kmix[j][i] for i in range(3) for j in range(3))
    Rs = trace_with(gi, R)
    if constraint_matter:
        rho = (Rs + trK * trK - KK) * (1.0 / (16.0 * math.pi))
        Si = []
        for i in range(3):
            e = _sum(Kmix[j][i].diff(j) for j in range(3))
            e = e + _sum(G[j][j][l] * Kmix[l][i] - G[l][j][i] * Kmix[j][l]
                         for j in range(3) for l in range(3))
            e = e - trK.diff(i)
            Si.append(e * (1.0 / (8.0 * math.pi)))
    else:
        rho = zero
        Si = [zero, zero, zero]
    if Sij is None:
        Sij = [[zero] * 3 for _ in range(3)]
    S = trace_with(gi, Sij)
    DDa = [[alpha.diff(i).diff(j) - _sum(G[k][i][j] * alpha.diff(k) for k in range(3))
            for j in range(3)] for i in range(3)]
    LbG = lie_sym(g, beta)
    LbK = lie_sym(K, beta)
    KKm = matmul(K, Kmix)
    gd = [[-2.0 * (alpha * K[i][j]) + LbG[i][j] for j in range(3)] for i in range(3)]
    Kd = [[-DDa[i][j] + alpha * (R[i][j] - 2.0 * KKm[i][j] + trK * K[i][j])
           - 8.0 * math.pi * (alpha * (Sij[i][j] - g[i][j] * (S - rho) * 0.5)) + LbK[i][j]
           for j in range(3)] for i in range(3)]

    chi = det3(g) ** (-1.0 / 3.0)
    chid = -(chi * trace_with(gi, gd)) * (1.0 / 3.0)
    gt = [[chi * g[i][j] for j in range(3)] for i in range(3)]
    gtd = [[chid * g[i][j] + chi * gd[i][j] for j in range(3)] for i in range(3)]
    gigd = matmul(matmul(gi, gd), gi)
    trKd = -trace_with(gigd, K) + trace_with(gi, Kd)
    out = {"chi": chid.v, "Khat": trKd.v, "Theta": np.zeros(shape),
           "alpha": np.zeros(shape)}
    for a, (i, j) in enumerate(SYM):
        out[FIELDS[1 + a]] = gtd[i][j].v
        Ad = chid * (K[i][j] - g[i][j] * trK * (1.0 / 3.0)) + chi * (
            Kd[i][j] - gd[i][j] * trK * (1.0 / 3.0) - g[i][j] * trKd * (1.0 / 3.0))
        out[FIELDS[8 + a]] = Ad.v
    # Gt^i = git^{jk} git^{il} Gt_{l jk};  d_t through the chain rule
    git = [[gi[i][j] / chi for j in range(3)] for i in range(3)]
    gitd = [[-_sum(git[i][a] * gtd[a][b] * git[b][j] for a in range(3) for b in range(3))
             for j in range(3)] for i in range(3)]
    for i in range(3):
        acc = None
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    low = (gt[k][l].diff(j) + gt[j][l].diff(k) - gt[j][k].diff(l)) * 0.5
                    lowd = (gtd[k][l].diff(j) + gtd[j][l].diff(k) - gtd[j][k].diff(l)) * 0.5
                    e = (gitd[j][k] * git[i][l] + git[j][k] * gitd[i][l]) * low \
                        + git[j][k] * git[i][l] * lowd
                    acc = e if acc is None else acc + e
        out[FIELDS[15 + i]] = acc.v
    for i in range(3):
        out[FIELDS[19 + i]] = np.zeros(shape)
    matter = [rho.v] + [s.v for s in Si] + [Sij[i][j].v for (i, j) in SYM]
    return out, [np.broadcast_to(m, shape).copy() for m in matter]


# --- exact spacetimes -------------------------------------------------------------

def _coords(X, Y, Z):
    return Jet.coord(0, X), Jet.coord(1, Y), Jet.coord(2, Z)


def kerr_schild_adm(X, Y, Z, M=1.0):
    """Schwarzschild in Kerr-Schild form: gamma = delta + 2H l l, H = M/r,
    alpha = (1+2H)^(-1/2), beta^i = 2H l^i / (1+2H); static, so
    K_ij = (D_i beta_j + D_j beta_i) / (2 alpha)."""
    x, y, z = _coords(X, Y, Z)
    r = jsqrt(x * x + y * y + z * z)
    H = M * r.recip()
    l = [x / r, y / r, z / r]
    g = [[(1.0 if i == j else 0.0) + 2.0 * (H * l[i] * l[j]) for j in range(3)]
         for i in range(3)]
    g = [[g[i][j] if isinstance(g[i][j], Jet) else Jet.const(g[i][j], X.shape)
          for j in range(3)] for i in range(3)]
    alpha = (1.0 + 2.0 * H) ** -0.5
    beta = [(2.0 * (H * l[i])) / (1.0 + 2.0 * H) for i in range(3)]
    gi = inv3(g)
    _, G = christoffel(g, gi)
    bl = [_sum(g[i][k] * beta[k] for k in range(3)) for i in range(3)]
    K = [[(bl[j].diff(i) + bl[i].diff(j) - 2.0 * _sum(G[k][i][j] * bl[k] for k in range(3)))
          / (2.0 * alpha) for j in range(3)] for i in range(3)]
    return g, K, alpha, beta


def kerr_schild(X, Y, Z, M=1.0):
    """(Z4c fields, d_t with frozen gauge, matter=0) for Kerr-Schild."""
    g, K, alpha, beta = kerr_schild_adm(X, Y, Z, M)
    u = z4c_from_adm(g, K, alpha, beta)
    dt, matter = adm_evolution(g, K, alpha, beta)
    return u, dt, matter


def generic_adm(X, Y, Z, seed=0):
    """Generic smooth ADM data: every metric, curvature, lapse, shift and
    stress component is a seeded plane wave of modest amplitude."""
    rng = np.random.default_rng(1234 + seed)
    x, y, z = _coords(X, Y, Z)

    def wave(a):
        amp = rng.uniform(-a, a)
        kx, ky, kz = rng.integers(1, 4, size=3) / 2.0
        ph = rng.uniform(-3, 3)
        return amp * jsin(kx * x + ky * y - kz * z + ph)

    g = [[None] * 3 for _ in range(3)]
    K = [[None] * 3 for _ in range(3)]
    S = [[None] * 3 for _ in range(3)]
    for (i, j) in SYM:
        gij = wave(0.15)
        if i == j:
            gij = gij + 1.0
        g[i][j] = g[j][i] = gij
        K[i][j] = K[j][i] = wave(0.2)
        S[i][j] = S[j][i] = wave(0.05)
    alpha = wave(0.2) + 1.0
    beta = [wave(0.2) for _ in range(3)]
    return g, K, alpha, beta, S


def generic_with_matter(X, Y, Z, seed=0):
    g, K, alpha, beta, S = generic_adm(X, Y, Z, seed)
    u = z4c_from_adm(g, K, alpha, beta)
    dt, matter = adm_evolution(g, K, alpha, beta, Sij=S, constraint_matter=True)
    return u, dt, matter


def gauge_wave(X, Y, Z, amp=0.1, direction="x"):
    """Gauge wave (harmonic slicing, zero shift), exact in time:
    'x' : H = 1 - A sin(2 pi (x - t)), gamma = diag(H, 1, 1), alpha = sqrt(H)
    'xy': H = 1 - A sin(2 pi (x + y) - 2 pi sqrt(2) t), gamma = delta + (H-1) n n,
          n = (1, 1, 0)/sqrt(2).
    Every field is a function of the phase only, so d_t = -(omega / k_x) d_x.
    Returns (Z4c fields, exact d_t of the Z4c fields)."""
    x, y, z = _coords(X, Y, Z)
    shape = X.shape
    if direction == "x":
        ph = 2.0 * math.pi * x
        omega, kx = 2.0 * math.pi, 2.0 * math.pi
        n = [1.0, 0.0, 0.0]
    else:
        ph = 2.0 * math.pi * (x + y)
        omega, kx = 2.0 * math.pi * math.sqrt(2.0), 2.0 * math.pi
        n = [1.0 / math.sqrt(2.0), 1.0 / math.sqrt(2.0), 0.0]
    H = 1.0 - amp * jsin(ph)
    dHdt = (omega * amp) * jcos(ph)       # d_t H at t = 0
    g = [[(H - 1.0) * (n[i] * n[j]) + (1.0 if i == j else 0.0) for j in range(3)]
         for i in range(3)]
    alpha = jsqrt(H)
    K = [[-(dHdt * (n[i] * n[j])) / (2.0 * alpha) for j in range(3)] for i in range(3)]
    zero = Jet.const(0.0, shape)
    beta = [zero, zero, zero]
    # fields as jets (values, and their x-derivative for the time derivative)
    gi = inv3(g)
    trK = trace_with(gi, K)
    chi = det3(g) ** (-1.0 / 3.0)
    gt = [[chi * g[i][j] for j in range(3)] for i in range(3)]
    git = [[gi[i][j] / chi for j in range(3)] for i in range(3)]
    _, up = christoffel(gt, git)
    fields = {"chi": chi, "Khat": trK, "Theta": zero, "alpha": alpha,
              "bx": zero, "by": zero, "bz": zero}
    for a, (i, j) in enumerate(SYM):
        fields[FIELDS[1 + a]] = gt[i][j]
        fields[FIELDS[8 + a]] = chi * (K[i][j] - g[i][j] * trK * (1.0 / 3.0))
    for i in range(3):
        fields[FIELDS[15 + i]] = trace_with(git, [[up[i][j][k] for k in range(3)]
                                                  for j in range(3)])
    u = {k: v.v for k, v in fields.items()}
    dt = {k: -(omega / kx) * v.diff(0).v for k, v in fields.items()}
    return u, dt
