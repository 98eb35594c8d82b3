"""Deterministic collision-probability (CP) model of one IUGKP iteration in 1D.

Test-side pin for the oracle.  For a slab of flat cells with isotropic,
uniform-in-cell emission, black walls with cosine-law emission and analog
collision tallies, the expected result of one particle iteration is exactly a
linear map built from the exponential integral E_3 (first-flight collision
probabilities of slab geometry).  This is the discrete form of the paper's
integral solution (Sec. 2: survival probability P_f, collision density P_c,
and the convex-combination form of the cell energies).

Notation: a_c = dx / lambda_c is the optical thickness of cell c,
lambda_c = |V_g| tau_c.  Real collisions follow the true optical depths
(delta tracking reproduces them, Sec. 3.2); candidate events in cell c are
1/r_c times the real ones, r_c = tau_min / tau_c.
"""
from __future__ import annotations

import numpy as np
from scipy.special import expn


def E3(x):
    return expn(3, np.asarray(x, dtype=np.float64))


def cp_1d(tau: np.ndarray, dx: float, vg: float = 1.0):
    """Return (K, Pw, Pesc, Pww).

    K[j, i]   : probability that a particle emitted uniformly/isotropically in cell j
                has its real collision in cell i;
    Pw[f, i]  : same for a cosine-law particle entering from wall f (0 left, 1 right);
    Pesc[j, f]: probability that a particle from cell j is absorbed by wall f;
    Pww[f, g] : wall f to wall g (g != f) without collision.
    """
    tau = np.asarray(tau, dtype=np.float64)
    n = tau.size
    a = dx / (vg * tau)
    cum = np.concatenate([[0.0], np.cumsum(a)])  # optical coordinate of face k
    K = np.zeros((n, n))
    for j in range(n):
        for i in range(n):
            if i == j:
                K[j, i] = 1.0 - (1.0 / a[j]) * (0.5 - E3(a[j]))
            else:
                lo, hi = (j, i) if j < i else (i, j)
                gap = cum[hi] - cum[lo + 1]
                K[j, i] = (1.0 / (2.0 * a[j])) * (E3(gap) - E3(gap + a[i]) - E3(gap + a[j])
                                                  + E3(gap + a[i] + a[j]))
    Pw = np.zeros((2, n))
    for i in range(n):
        Pw[0, i] = 2.0 * (E3(cum[i]) - E3(cum[i + 1]))
        Pw[1, i] = 2.0 * (E3(cum[n] - cum[i + 1]) - E3(cum[n] - cum[i]))
    Pesc = np.zeros((n, 2))
    for j in range(n):
        Pesc[j, 0] = (1.0 / (2.0 * a[j])) * (E3(cum[j]) - E3(cum[j + 1]))
        Pesc[j, 1] = (1.0 / (2.0 * a[j])) * (E3(cum[n] - cum[j + 1]) - E3(cum[n] - cum[j]))
    Pww = np.zeros((2, 2))
    Pww[0, 1] = Pww[1, 0] = 2.0 * E3(cum[n])
    return K, Pw, Pesc, Pww


class Slab:
    """Expected one-iteration map of a 1D workload, in floating point energy units."""

    def __init__(self, w):
        self.w = w
        self.tau = np.asarray(w.tau, dtype=np.float64)
        self.tau_min = self.tau.min()
        self.lam_min = w.vg * self.tau_min
        self.r = self.tau_min / self.tau
        self.V = w.dx * w.dy
        self.K, self.Pw, self.Pesc, self.Pww = cp_1d(self.tau, w.dx, w.vg)
        self.Ew = w.cv * (np.asarray(w.wall_T) - w.t_ref)
        self.Gw = self.Ew * self.lam_min * 1.0 / 4.0

    def cell_emission(self, E):
        return self.r * np.asarray(E) * self.V

    def expected_D(self, Gc):
        return Gc @ self.K + self.Gw @ self.Pw

    def expected_B(self, Gc):
        return Gc @ self.Pesc + self.Gw @ self.Pww

    def expected_W(self, Gc):
        return self.expected_D(Gc) / self.r

    def step(self, E):
        """E^{n+1} = E[W]/V for emission from E (no Newton)."""
        return self.expected_W(self.cell_emission(E)) / self.V

    def fixed_point(self, source=None):
        """Steady state of the re-emission map G -> D + G_src (G_src = S V tau_min
        per iteration, zero without a source), returned as E = W/V."""
        n = self.tau.size
        A = np.eye(n) - self.K.T
        Gs = np.zeros(n) if source is None else np.asarray(source) * self.V * self.tau_min
        G = np.linalg.solve(A, self.Gw @ self.Pw + Gs)
        return self.expected_W(G) / self.V, G

    def heat_flux_left(self, G):
        """Net energy flux through the left wall face per unit area and time."""
        absorbed = self.expected_B(G)[0]
        return (self.Gw[0] - absorbed) / (1.0 * self.tau_min)

    def psi(self):
        """Heat-flux ratio q / (|V_g| (E_H - E_L) / 4) at the fixed point."""
        _, G = self.fixed_point()
        return self.heat_flux_left(G) / (self.w.vg * (self.Ew[0] - self.Ew[1]) / 4.0)

    def variance_D(self, Gc, n_per):
        """Variance of the D tally for one iteration (multinomial per emitter)."""
        var = np.zeros(self.tau.size)
        for j, g in enumerate(Gc):
            q = g / n_per
            p = self.K[j]
            var += n_per * q * q * p * (1 - p)
        for f in range(2):
            q = self.Gw[f] / n_per
            p = self.Pw[f]
            var += n_per * q * q * p * (1 - p)
        return var

    def variance_W(self, Gc, n_per):
        """Variance of W for delta tracking: per-emitter variance of sum over
        candidate events (geometric count 1/r per real collision in a cell)."""
        # For each particle, W contribution to cell i is q * N_i with N_i the number of
        # candidate events in i; E[N_i^2] <= E[N_i] (2/r_i - 1) for the geometric count
        # when the real collision happens in i; used only as an upper bound.
        var = np.zeros(self.tau.size)
        for j, g in enumerate(Gc):
            q = g / n_per
            m = self.K[j] / self.r
            var += n_per * q * q * m * (2.0 / self.r)
        for f in range(2):
            q = self.Gw[f] / n_per
            m = self.Pw[f] / self.r
            var += n_per * q * q * m * (2.0 / self.r)
        return var


def d_eff(lam: float, delta: float, tol: float = 1e-18) -> float:
    """Per-iteration diffusion coefficient of the flat-cell 1D kernel:
    half the second moment of the cell-to-cell jump,
    D = sum_{m>=1} m^2 delta^2 P_m  =  (lam delta / 2) (1/2 + 2 sum_{j>=1} E_3(j delta/lam)).
    Tends to lam^2/3 for lam >> delta and to lam delta / 4 for lam << delta."""
    a = delta / lam
    jmax = int(np.ceil(60.0 / a)) + 2
    j = np.arange(1, jmax + 1, dtype=np.float64)
    s = np.sum(E3(j * a)[::-1])
    return (lam * delta / 2.0) * (0.5 + 2.0 * s)


def d_eff_second_moment(lam: float, delta: float, mmax: int = 20000) -> float:
    """Same quantity from its definition, sum_m m^2 delta^2 P_m (slower; used to check d_eff)."""
    a = delta / lam
    m = np.arange(1, mmax + 1, dtype=np.float64)
    P = (1.0 / (2.0 * a)) * (E3((m - 1) * a) - 2.0 * E3(m * a) + E3((m + 1) * a))
    return float(np.sum((m * m * delta * delta * P)[::-1]))


def newton_matrix_1d(n: int, dx: float, lam: np.ndarray, D: np.ndarray) -> np.ndarray:
    """Dense conservative 3-point operator -d/dx(D d/dx) with Robin walls
    (extrapolation distance 2 lam / 3), per-iteration units."""
    A = np.zeros((n, n))
    for k in range(n + 1):
        if k == 0 or k == n:
            c = 0 if k == 0 else n - 1
            g = D[c] / (dx * (dx / 2 + 2 * lam[c] / 3))
            A[c, c] += g
        else:
            a, b = D[k - 1], D[k]
            g = 2 * a * b / (a + b) / dx ** 2
            A[k - 1, k - 1] += g
            A[k, k] += g
            A[k - 1, k] -= g
            A[k, k - 1] -= g
    return A


def dsa_spectral_radius(w, D=None) -> float:
    """Spectral radius of the deterministic accelerated iteration
    E -> E_half + A^{-1} (E_half - E), E_half = K-map(E) (error propagation)."""
    s = Slab(w)
    n = w.nx
    lam = w.vg * s.tau
    if D is None:
        D = np.array([d_eff(l, w.dx) for l in lam])
    A = newton_matrix_1d(n, w.dx, lam, D)
    M = (s.K.T * (s.r[None, :] * s.V)) / (s.r[:, None] * s.V)   # E -> E_half (homogeneous part)
    I = np.eye(n)
    T = M + np.linalg.solve(A, M - I)
    return float(np.max(np.abs(np.linalg.eigvals(T))))


def bands_fixed_point_1d(w, source=None):
    """Expected steady state of the multi-band iteration on a 1D film with the
    exact E_3 kernels of every band: the absorbed rate R solves R = R M + b with
    M[e, i] = sum_k p_k(e) K_k[e, i] (p_k the equilibrium spectrum C_k/tau_k,
    normalised), b = sum_k (Gw_k Pw_k) / tau*_k + S V; then E = sum_k W_k / V
    with E[W_k] = E[D_k] / (tau*_k / tau_k).  Returns (E, R)."""
    K, n = int(w.n_bands), w.nx
    tau = np.asarray(w.tau, dtype=np.float64).reshape(K, n)
    C = np.asarray(w.band_C, dtype=np.float64)
    v = np.asarray(w.band_vg, dtype=np.float64)
    V = w.dx * w.dy
    ts = tau.min(axis=1)
    den = (C[:, None] / tau).sum(axis=0)
    M = np.zeros((n, n))
    b = np.zeros(n) if source is None else np.asarray(source) * V
    Ew = np.asarray(w.wall_T) - w.t_ref
    mats = []
    for k in range(K):
        Kk, Pw, _, _ = cp_1d(tau[k], w.dx, v[k])
        mats.append((Kk, Pw))
        pk = (C[k] / tau[k]) / den
        M += pk[:, None] * Kk
        Gw = C[k] * Ew * v[k] * ts[k] * 1.0 / 4.0
        b += (Gw @ Pw) / ts[k]
    R = np.linalg.solve((np.eye(n) - M).T, b)
    E = np.zeros(n)
    for k in range(K):
        Kk, Pw = mats[k]
        Gk = ts[k] * ((C[k] / tau[k]) / den) * R
        Gw = C[k] * Ew * v[k] * ts[k] / 4.0
        Dk = Gk @ Kk + Gw @ Pw
        E += Dk / (ts[k] / tau[k])
    return E / V, R


# ------------------------------------------------------------------ 2D flat cells
# A particle emitted uniformly in a square cell with a 3D-isotropic direction
# and an exponential path of mean lambda (cell units) moves in the plane by a
# radially symmetric displacement whose radial density is the Bickley form
#     f(rho) = (1/lambda) int_0^{pi/2} exp(-rho / (lambda sin th)) d th
# (the in-plane length is the 3D length times sin th).  A uniform start in the
# cell and binning of the end point by cell make the cell-to-cell probability
# the expectation of the 2D tent T(u - m) T(v - n) over the displacement (u, v).
# In a convex domain a straight flight between two interior cells never leaves
# it, so the expected one-iteration map of a uniform-tau square mesh is this
# infinite-medium kernel restricted to the mesh (walls absorb the rest).

def bickley_density(rho: np.ndarray, lam: float, nth: int = 400) -> np.ndarray:
    x, w = np.polynomial.legendre.leggauss(nth)
    th = (x + 1.0) * np.pi / 4.0
    w = w * np.pi / 4.0
    s = np.sin(th)
    return (np.exp(-np.asarray(rho)[:, None] / (lam * s[None, :])) @ w) / lam


def transfer_2d_real(lam: float, R: int, panels: int = 300, gauss: int = 10,
                     nphi: int = 8192) -> np.ndarray:
    """P[m, n], 0 <= m, n <= R: probability of a displacement by (m, n) cells,
    by quadrature of the radial density (Gauss panels in rho, midpoint in the
    angle) and bilinear (tent) binning."""
    rmax = min(40.0 * lam + 2.0, np.hypot(R, R) + 2.0)
    edges = np.linspace(0.0, rmax, panels + 1)
    x, w = np.polynomial.legendre.leggauss(gauss)
    half = (edges[1:] - edges[:-1])[:, None] / 2.0
    rho = ((edges[1:] + edges[:-1])[:, None] / 2.0 + half * x[None, :]).ravel()
    wr = (half * w[None, :]).ravel()
    fr = bickley_density(rho, lam) * wr
    phi = (np.arange(nphi) + 0.5) * 2.0 * np.pi / nphi
    P = np.zeros((R + 3, R + 3))
    for i0 in range(0, rho.size, 200):
        r = rho[i0:i0 + 200, None]
        wt = np.broadcast_to(fr[i0:i0 + 200, None] / nphi, (r.shape[0], nphi))
        u = np.abs(r * np.cos(phi)[None, :])
        v = np.abs(r * np.sin(phi)[None, :])
        mu, mv = np.floor(u).astype(int), np.floor(v).astype(int)
        fu, fv = u - mu, v - mv
        for dm, wu in ((0, 1.0 - fu), (1, fu)):
            for dn, wv in ((0, 1.0 - fv), (1, fv)):
                mm, nn = mu + dm, mv + dn
                ok = (mm <= R + 2) & (nn <= R + 2)
                np.add.at(P, (mm[ok], nn[ok]), (wt * wu * wv)[ok])
    # |u| and |v| fold both signs of a nonzero offset onto one entry
    P[1:, :] /= 2.0
    P[:, 1:] /= 2.0
    return P[:R + 1, :R + 1]


def transfer_2d_fourier(lam: float, R: int, nk: int = 256, aliases: int = 24) -> np.ndarray:
    """The same P[m, n] from its discrete-time Fourier transform: the
    characteristic function of a 3D-isotropic exponential flight at an in-plane
    wave vector xi is arctan(lambda |xi|) / (lambda |xi|); the tent contributes
    sinc^2 per axis; aliases xi = k + 2 pi j are summed for |j| <= aliases
    (accurate when lambda is not small against a cell)."""
    k = 2.0 * np.pi * (np.arange(nk) - nk // 2) / nk
    KX, KY = np.meshgrid(k, k, indexing="ij")
    Kh = np.zeros_like(KX)
    for jx in range(-aliases, aliases + 1):
        ax = KX + 2.0 * np.pi * jx
        sx = np.sinc(ax / (2.0 * np.pi)) ** 2
        for jy in range(-aliases, aliases + 1):
            ay = KY + 2.0 * np.pi * jy
            z = lam * np.hypot(ax, ay)
            zs = np.where(z > 0.0, z, 1.0)
            Kh += np.where(z > 0.0, np.arctan(zs) / zs, 1.0) * sx * np.sinc(ay / (2.0 * np.pi)) ** 2
    P = np.real(np.fft.ifft2(np.fft.ifftshift(Kh)))
    return P[:R + 1, :R + 1]


def transfer_2d(lam: float, R: int) -> np.ndarray:
    return transfer_2d_real(lam, R) if lam <= 1.0 else transfer_2d_fourier(lam, R)


def dense_transfer_2d(nx: int, ny: int, lam: float) -> np.ndarray:
    """Expected one-iteration map E -> E_half of a uniform-tau nx x ny cavity
    (cells c = ix + nx iy; lam in cell units, square cells)."""
    P = transfer_2d(lam, max(nx, ny) - 1)
    ix = np.tile(np.arange(nx), ny)
    iy = np.repeat(np.arange(ny), nx)
    return P[np.abs(ix[:, None] - ix[None, :]), np.abs(iy[:, None] - iy[None, :])]


def flat_cell_jump_1d(lam: float, m: int) -> float:
    """Probability of a 1D flat-cell jump by m >= 0 cells (lam in cell units)."""
    a = 1.0 / lam
    if m == 0:
        return float(1.0 - lam * (0.5 - E3(a)))
    return float((lam / 2.0) * (E3((m - 1) * a) - 2.0 * E3(m * a) + E3((m + 1) * a)))
