"""Independent analytic restatements used to pin the oracle (numpy only).

Nothing here calls the oracle or the HIP library. Each function states a
definition from the paper (coordinates, rescaled basis) or a closed form that
follows from it (Brill-Lindquist right-hand sides, textbook Ricci tensor of a
given metric, pure-gauge shift right-hand sides).
"""
import numpy as np

SINH_SPHERICAL, SINH_CYLINDRICAL, SPHERICAL = 0, 1, 2
NGF = 24
GF_NAMES = ["aDD00", "aDD01", "aDD02", "aDD11", "aDD12", "aDD22", "alpha",
            "betU0", "betU1", "betU2", "cf", "hDD00", "hDD01", "hDD02", "hDD11",
            "hDD12", "hDD22", "lambdaU0", "lambdaU1", "lambdaU2", "trK",
            "vetU0", "vetU1", "vetU2"]
GF = {n: i for i, n in enumerate(GF_NAMES)}
SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


# ---- grid and coordinates (Sec. 3 cell centring; Eqs. 18-20, 22) ---------
def domain(coord):
    if coord == SINH_CYLINDRICAL:
        return [(0.0, 1.0), (-np.pi, np.pi), (-1.0, 1.0)]
    return [(0.0, 1.0), (0.0, np.pi), (-np.pi, np.pi)]


def axes(coord, N, ng=3):
    out = []
    for d, (lo, hi) in enumerate(domain(coord)):
        dx = (hi - lo) / N[d]
        j = np.arange(N[d] + 2 * ng)
        out.append(lo + (j - ng + 0.5) * dx)
    return out


def sinh_map(x, A, w):
    return A * np.sinh(x / w) / np.sinh(1.0 / w)


def mesh(coord, N, ampl, sinhw, ng=3):
    """Logical coordinates, Cartesian position and rescaled basis at every
    point (ghosts included). Arrays have shape (n2, n1, n0[, 3])."""
    a0, a1, a2 = axes(coord, N, ng)
    X2, X1, X0 = np.meshgrid(a2, a1, a0, indexing="ij")
    if coord == SINH_CYLINDRICAL:
        rho = sinh_map(X0, ampl[0], sinhw[0])
        z = sinh_map(X2, ampl[2], sinhw[2])
        ph = X1
        x = np.stack([rho * np.cos(ph), rho * np.sin(ph), z], axis=-1)
        zero = np.zeros_like(ph)
        one = np.ones_like(ph)
        e0 = np.stack([np.cos(ph), np.sin(ph), zero], -1)
        e1 = np.stack([-np.sin(ph), np.cos(ph), zero], -1)
        e2 = np.stack([zero, zero, one], -1)
    else:
        r = ampl[0] * X0 if coord == SPHERICAL else sinh_map(X0, ampl[0], sinhw[0])
        th, ph = X1, X2
        x = np.stack([r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph),
                      r * np.cos(th)], axis=-1)
        e0 = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1)
        e1 = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)], -1)
        e2 = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], -1)
    E = np.stack([e0, e1, e2], axis=-2)  # E[..., i, a] = component a of e~_(i)
    return (X0, X1, X2), x, E


def to_frame_vec(E, V):
    """Rescaled (orthonormal-frame) components of a Cartesian vector field."""
    return np.einsum("...ia,...a->...i", E, V)


def to_frame_sym(E, T):
    """Rescaled components of a Cartesian covariant symmetric tensor."""
    return np.einsum("...ia,...jb,...ab->...ij", E, E, T)


# ---- Brill-Lindquist (conformally flat, time symmetric) -------------------
def bl_psi(x, masses, pos):
    psi = np.ones(x.shape[:-1])
    grad = np.zeros(x.shape)
    for m, c in zip(masses, pos):
        d = x - np.asarray(c, dtype=float)
        r = np.sqrt(np.sum(d * d, axis=-1))
        psi += m / (2.0 * r)
        grad += (-m / (2.0 * r ** 3))[..., None] * d
    return psi, grad


def bl_state(coord, N, ampl, sinhw, masses, pos, lapse_kind=0, ng=3):
    """State array (24, n2, n1, n0) of BL data evaluated at every point."""
    _, x, _ = mesh(coord, N, ampl, sinhw, ng)
    psi, _ = bl_psi(x, masses, pos)
    y = np.zeros((NGF,) + psi.shape)
    y[GF["cf"]] = psi ** -2
    y[GF["alpha"]] = psi ** -2 if lapse_kind == 0 else 1.0
    return y


def bl_rhs_closed_form(coord, N, ampl, sinhw, masses, pos, ng=3):
    """Continuum right-hand sides of BL data with alpha = psi^-2, beta = 0:
    d_t K = -2 psi^-8 |grad psi|^2,
    d_t a_ij (frame) = -8 psi^-8 (d_i psi d_j psi - delta_ij |grad psi|^2 / 3),
    every other variable 0."""
    _, x, E = mesh(coord, N, ampl, sinhw, ng)
    psi, g = bl_psi(x, masses, pos)
    g2 = np.sum(g * g, axis=-1)
    out = np.zeros((NGF,) + psi.shape)
    out[GF["trK"]] = -2.0 * psi ** -8 * g2
    T = -8.0 * psi[..., None, None] ** -8 * (g[..., :, None] * g[..., None, :]
                                             - np.eye(3) * (g2 / 3.0)[..., None, None])
    Tf = to_frame_sym(E, T)
    for c, (i, j) in enumerate(SYM):
        out[GF["aDD00"] + c] = Tf[..., i, j]
    return out


# ---- a curved conformal metric and its textbook Ricci tensor --------------
def gaussian_metric(x, amp, M, c, sigma):
    """gbar_ab = delta_ab + amp G(x) M_ab, G = exp(-|x-c|^2/sigma^2), with
    first and second Cartesian derivatives."""
    d = x - np.asarray(c, dtype=float)
    G = np.exp(-np.sum(d * d, -1) / sigma ** 2)
    Gd = (-2.0 / sigma ** 2) * d * G[..., None]
    Gdd = (4.0 / sigma ** 4) * d[..., :, None] * d[..., None, :] * G[..., None, None] \
        - (2.0 / sigma ** 2) * np.eye(3) * G[..., None, None]
    M = np.asarray(M, dtype=float)
    g = np.eye(3) + amp * G[..., None, None] * M
    dg = amp * np.einsum("ab,...c->...abc", M, Gd)          # d_c g_ab
    ddg = amp * np.einsum("ab,...cd->...abcd", M, Gdd)      # d_c d_d g_ab
    return g, dg, ddg


def christoffel_and_ricci(g, dg, ddg):
    """Cartesian Christoffel symbols Gam[a,b,c] = Gamma^a_bc, the contracted
    Lam^a = g^bc Gamma^a_bc, and the Ricci tensor
    R_bd = d_a Gam^a_bd - d_d Gam^a_ba + Gam^a_ae Gam^e_bd - Gam^a_de Gam^e_ba."""
    gi = np.linalg.inv(g)
    # lowered Gamma_dbc = 1/2 (d_b g_dc + d_c g_db - d_d g_bc)
    Gl = 0.5 * (np.einsum("...dcb->...dbc", dg) + dg - np.einsum("...bcd->...dbc", dg))
    Gam = np.einsum("...ad,...dbc->...abc", gi, Gl)
    dgi = -np.einsum("...ap,...pqe,...qd->...ade", gi, dg, gi)      # d_e g^ad
    dGl = 0.5 * (np.einsum("...dcbe->...dbce", ddg) + np.einsum("...dbce->...dbce", ddg)
                 - np.einsum("...bcde->...dbce", ddg))             # d_e Gamma_dbc
    dGam = np.einsum("...ade,...dbc->...abce", dgi, Gl) + np.einsum("...ad,...dbce->...abce", gi, dGl)
    R = (np.einsum("...abda->...bd", dGam) - np.einsum("...abad->...bd", dGam)
         + np.einsum("...aae,...ebd->...bd", Gam, Gam) - np.einsum("...ade,...eba->...bd", Gam, Gam))
    Lam = np.einsum("...bc,...abc->...a", gi, Gam)
    return Gam, Lam, R


# ---- pure-gauge shift on flat space ---------------------------------------
def gauge_field(x, amp, c, sigma, V, L):
    """xi^a(x) = amp G(x) (V^a + L^a_b (x-c)^b) and its first and second
    Cartesian derivatives dxi[a,b] = d_b xi^a, ddxi[a,b,c] = d_b d_c xi^a."""
    d = x - np.asarray(c, dtype=float)
    G = np.exp(-np.sum(d * d, -1) / sigma ** 2)
    Gd = (-2.0 / sigma ** 2) * d * G[..., None]
    Gdd = (4.0 / sigma ** 4) * d[..., :, None] * d[..., None, :] * G[..., None, None] \
        - (2.0 / sigma ** 2) * np.eye(3) * G[..., None, None]
    V = np.asarray(V, dtype=float)
    L = np.asarray(L, dtype=float)
    P = V + np.einsum("ab,...b->...a", L, d)              # polynomial part
    xi = amp * G[..., None] * P
    dxi = amp * (np.einsum("...a,...b->...ab", P, Gd) + G[..., None, None] * L)
    ddxi = amp * (np.einsum("...a,...bc->...abc", P, Gdd)
                  + np.einsum("ab,...c->...abc", L, Gd) + np.einsum("ac,...b->...abc", L, Gd))
    return xi, dxi, ddxi


def diag_christoffel(coord, X0, X1, X2, ampl, sinhw):
    """Gammahat^i_jk of the diagonal reference metric gammahat_ii = S_i^2:
    Gammahat^i_ij = Gammahat^i_ji = d_j S_i / S_i, Gammahat^i_jj = -S_j d_i S_j / S_i^2
    (j != i), all others 0; S and dS restated from the coordinate maps."""
    shp = X0.shape
    S = np.zeros(shp + (3,))
    dS = np.zeros(shp + (3, 3))  # dS[..., i, k] = d_k S_i
    if coord == SINH_CYLINDRICAL:
        A, w = ampl[0], sinhw[0]
        s = np.sinh(1.0 / w)
        rho, rp, rpp = A * np.sinh(X0 / w) / s, A * np.cosh(X0 / w) / (w * s), A * np.sinh(X0 / w) / (w * w * s)
        Az, wz = ampl[2], sinhw[2]
        sz = np.sinh(1.0 / wz)
        zp, zpp = Az * np.cosh(X2 / wz) / (wz * sz), Az * np.sinh(X2 / wz) / (wz * wz * sz)
        S[..., 0], S[..., 1], S[..., 2] = rp, rho, zp
        dS[..., 0, 0], dS[..., 1, 0], dS[..., 2, 2] = rpp, rp, zpp
    else:
        if coord == SPHERICAL:
            r, rp, rpp = ampl[0] * X0, ampl[0] * np.ones(shp), np.zeros(shp)
        else:
            A, w = ampl[0], sinhw[0]
            s = np.sinh(1.0 / w)
            r, rp, rpp = A * np.sinh(X0 / w) / s, A * np.cosh(X0 / w) / (w * s), A * np.sinh(X0 / w) / (w * w * s)
        st, ct = np.sin(X1), np.cos(X1)
        S[..., 0], S[..., 1], S[..., 2] = rp, r, r * st
        dS[..., 0, 0] = rpp
        dS[..., 1, 0] = rp
        dS[..., 2, 0] = rp * st
        dS[..., 2, 1] = r * ct
    Gam = np.zeros(shp + (3, 3, 3))
    for i in range(3):
        for j in range(3):
            Gam[..., i, i, j] = dS[..., i, j] / S[..., i]
            Gam[..., i, j, i] = dS[..., i, j] / S[..., i]
        for j in range(3):
            if j != i:
                Gam[..., i, j, j] = -S[..., j] * dS[..., j, i] / S[..., i] ** 2
    return S, Gam


# ---- refinement helpers ---------------------------------------------------
def common_points(Nc, ng=3, ratio=3):
    """Index arrays (coarse, fine) of coarse interior points that are also
    fine-grid points under refinement by `ratio` (odd) in each direction
    whose ratio entry > 1."""
    out_c, out_f = [], []
    for d in range(3):
        r = ratio[d] if isinstance(ratio, (tuple, list)) else ratio
        jc = np.arange(Nc[d])
        out_c.append(jc + ng)
        out_f.append(r * jc + (r - 1) // 2 + ng)
    return out_c, out_f


# ---- Schwarzschild in Kerr-Schild coordinates (stationary) -----------------
def kerr_schild(x, M, c):
    """Schwarzschild of mass M centred at c in Kerr-Schild coordinates:
    gamma_ij = delta_ij + 2 M d_i d_j / r^3, alpha = (1 + 2M/r)^-1/2,
    beta^i = 2 M d_i / (r (r + 2M)), with d = x - c, r = |d|. Returns the
    physical metric, lapse, shift, their first Cartesian derivatives, and
    K_ij from d_t gamma_ij = 0 = -2 alpha K_ij + D_i beta_j + D_j beta_i."""
    d = x - np.asarray(c, dtype=float)
    r = np.sqrt(np.sum(d * d, -1))
    I3 = np.eye(3)
    dd = d[..., :, None] * d[..., None, :]
    gam = I3 + 2.0 * M * dd / r[..., None, None] ** 3
    # d_k (d_i d_j / r^3) = (delta_ik d_j + d_i delta_jk)/r^3 - 3 d_i d_j d_k / r^5
    dgam = 2.0 * M * ((np.einsum("ik,...j->...ijk", I3, d) + np.einsum("jk,...i->...ijk", I3, d))
                      / r[..., None, None, None] ** 3
                      - 3.0 * np.einsum("...ij,...k->...ijk", dd, d) / r[..., None, None, None] ** 5)
    alpha = (1.0 + 2.0 * M / r) ** -0.5
    dalpha = M * d * (alpha ** 3 / r ** 3)[..., None]
    gfun = 1.0 / (r * r + 2.0 * M * r)
    dgfun = -(2.0 * r + 2.0 * M)[..., None] * (d / r[..., None]) * (gfun ** 2)[..., None]
    beta = 2.0 * M * d * gfun[..., None]
    dbeta = 2.0 * M * (I3 * gfun[..., None, None] + np.einsum("...i,...k->...ik", d, dgfun))  # [i,k] = d_k beta^i
    gi = np.linalg.inv(gam)
    Gl = 0.5 * (np.einsum("...dcb->...dbc", dgam) + dgam - np.einsum("...bcd->...dbc", dgam))
    Gam = np.einsum("...ad,...dbc->...abc", gi, Gl)
    betaD = np.einsum("...jk,...k->...j", gam, beta)
    dbetaD = np.einsum("...jki,...k->...ij", dgam, beta) + np.einsum("...jk,...ki->...ij", gam, dbeta)  # [i,j] = d_i beta_j
    Dbeta = dbetaD - np.einsum("...kij,...k->...ij", Gam, betaD)
    Kij = (Dbeta + np.swapaxes(Dbeta, -1, -2)) / (2.0 * alpha[..., None, None])
    return dict(gam=gam, dgam=dgam, alpha=alpha, dalpha=dalpha, beta=beta, dbeta=dbeta, K=Kij,
                r=r, gi=gi)
