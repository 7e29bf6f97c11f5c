"""Analytic radiation force and torque on circular cylinders (TM^z).

TEST INFRASTRUCTURE ONLY: a validator for the FP64 lattice oracle, used by the
test-suite and by the script that writes the stored analytic tables.

Everything here follows arXiv 2509.22308 in the body frame of the paper:

* Sec. II, Eq. (incident field): E^I = sum_m alpha_m (-j)^m J_m(k0 r) cos m(phi - phi0),
  i.e. exp(-j k0 r cos(phi - phi0)); with the time factor exp(-j omega t)
  of Eq. (scattered field) this wave travels towards the body angle phi0 + pi.
* Sec. II, Eq. (scattered field): E^S = sum_m [B_m cos m phi + D_m sin m phi] H_m(k0 r).
* Sec. II.B, Eqs. (drag), (lift), (Torque): the time-averaged Maxwell stress
  integrated over r = a, projected on the lab axes x = body angle phi0 + pi,
  y = body angle phi0 + 3 pi / 2; normalised by F0 = pi a eps0 E0^2 / 4 and
  M0 = 2 F0 a (Sec. II.B).
* Sec. IV.A, Eqs. (constants_Bm_Dm), (integral equation), (discrete / matrix
  integral equation), (Fx), (Fy), (U), (V), (Torque), (coefficients): the
  metallo-dielectric Janus cylinder (region II = eps_r1 on body angles (0, pi),
  region III = PEC on (pi, 2 pi)).

Units: eps0 = mu0 = 1, E0 = 1, so omega = k0.

Numerics (the paper does not give N or the mode cut-off): the kernel of the
integral equation has rank <= 2M + 1 for M modes, so M >= (N - 1)/2 is needed;
we take M = N - 1.  Bessel ratios come from recurrences so that orders far
above the argument neither overflow nor underflow.  The discrete solution
converges like N^(-p) with p ~ 4/3 (edge singularity at the PEC/dielectric
junction), hence ``mdjc_forces_extrapolated`` applies Richardson extrapolation
over N, 2N - 1, 4N - 3.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def alpha(m):
    m = np.asarray(m)
    return np.where(m == 0, 1.0, 2.0)


def _hankel_ratios(z: float, M: int):
    """H_m'(z)/H_m(z) and 1/H_m(z) for m = 0..M, H = H^(1), real z > 0.

    Forward recurrence on s_m = H_m / H_{m-1} (stable: Y_m dominates):
    H_{m+1} = (2m/z) H_m - H_{m-1}.
    """
    h0 = special.hankel1(0, z)
    h1 = special.hankel1(1, z)
    s = np.empty(M + 2, dtype=complex)
    s[1] = h1 / h0
    for m in range(1, M + 1):
        s[m + 1] = 2.0 * m / z - 1.0 / s[m]
    hr = np.empty(M + 1, dtype=complex)
    hr[0] = -h1 / h0
    m = np.arange(1, M + 1)
    hr[1:] = 1.0 / s[1:M + 1] - m / z
    inv = np.empty(M + 1, dtype=complex)
    inv[0] = 1.0 / h0
    with np.errstate(under="ignore"):
        for k in range(1, M + 1):
            inv[k] = inv[k - 1] / s[k]
    return hr, inv


def _bessel_j_ratio(z: float, M: int):
    """J_m'(z)/J_m(z) for m = 0..M by backward recurrence on r_m = J_{m-1}/J_m."""
    start = M + 40 + int(2 * z)
    r = 2.0 * start / z
    out = np.empty(M + 2)
    for m in range(start, 0, -1):
        r_new = 2.0 * m / z - 1.0 / r          # r_m from r_{m+1}
        if m <= M + 1:
            out[m] = r_new
        r = r_new
    jr = np.empty(M + 1)
    # J_0'/J_0 = -J_1/J_0 = -1/r_1
    jr[0] = -1.0 / out[1]
    m = np.arange(1, M + 1)
    jr[1:] = out[1:M + 1] - m / z
    return jr


def _bessel_j(z: float, M: int):
    """J_m(z) and J_m'(z) for m = 0..M (underflow to 0 far above z is harmless here)."""
    m = np.arange(M + 1)
    with np.errstate(under="ignore"):
        j = special.jv(m, z)
        jp = special.jvp(m, z)
    return j, jp


def incident_coeffs(x: float, phi0: float, M: int):
    """Full-circle Fourier coefficients of the incident field on r = a."""
    m = np.arange(M + 1)
    j, jp = _bessel_j(x, M)
    base = alpha(m) * (-1j) ** m
    return base * j * np.cos(m * phi0), base * j * np.sin(m * phi0), base * jp * np.cos(m * phi0), base * jp * np.sin(m * phi0)


def _total_from_scattering(x: float, phi0: float, M: int, b_cos, b_sin):
    """C, S, C', S' of Eq. (coefficients) given B_m (b_cos) and D_m (b_sin)."""
    hr, inv = _hankel_ratios(x, M)
    with np.errstate(over="ignore", invalid="ignore"):
        h = 1.0 / inv
    ic, is_, icp, isp = incident_coeffs(x, phi0, M)
    # B_m H_m and B_m H_m' without forming H_m for large m
    bh_c = np.where(np.abs(b_cos) > 0, b_cos * h, 0.0)
    bh_s = np.where(np.abs(b_sin) > 0, b_sin * h, 0.0)
    return ic + bh_c, is_ + bh_s, icp + bh_c * hr, isp + bh_s * hr


def mie_coeffs(x: float, eps: float, phi0: float = 0.0, M: int | None = None):
    """Homogeneous dielectric cylinder (TM): C, S, C', S' on r = a.

    Continuity of E_z and dE_z/dr at r = a with the interior J_m(n k0 r) series
    gives the scattered fraction b_m of each incident partial wave:
    b_m = [n J_m'(nx) J_m(x) - J_m(nx) J_m'(x)] / [J_m(nx) H_m'(x) - n J_m'(nx) H_m(x)].
    """
    if M is None:
        M = int(x * math.sqrt(eps) + 30)
    n = math.sqrt(eps)
    m = np.arange(M + 1)
    j, jp = _bessel_j(x, M)
    jn, jnp = _bessel_j(n * x, M)
    h = special.hankel1(m, x)
    hp = special.h1vp(m, x)
    b = (n * jnp * j - jn * jp) / (jn * hp - n * jnp * h)
    base = alpha(m) * (-1j) ** m
    return _total_from_scattering(x, phi0, M, base * b * np.cos(m * phi0), base * b * np.sin(m * phi0))


def pec_coeffs(x: float, phi0: float = 0.0, M: int | None = None):
    """Homogeneous PEC cylinder (TM): E_z = 0 on r = a, b_m = -J_m(x)/H_m(x)."""
    if M is None:
        M = int(x + 30)
    m = np.arange(M + 1)
    j, _ = _bessel_j(x, M)
    b = -j / special.hankel1(m, x)
    base = alpha(m) * (-1j) ** m
    return _total_from_scattering(x, phi0, M, base * b * np.cos(m * phi0), base * b * np.sin(m * phi0))


def mie_te_coeffs(x: float, eps: float, phi0: float = 0.0, M: int | None = None):
    """Homogeneous dielectric cylinder, TE^z (Hz along the axis): C, S, C', S'
    of the total Hz on r = a.

    The incident Hz has the series of Eq. (incident field) (impedance 1, so
    |Hz^I| = E0).  Continuity of Hz and of E_phi = (j / (k0 eps)) dHz/dr at
    r = a with the interior J_m(n k0 r) series gives
    b_m = [J_m'(nx) J_m(x) - n J_m(nx) J_m'(x)] / [n J_m(nx) H_m'(x) - J_m'(nx) H_m(x)].
    The stress tensor is symmetric in E and H, and E (TE) is the curl of Hz
    up to a sign, as H (TM) is the curl of Ez: forces_closed_form and
    far_intensity apply to these coefficients unchanged.
    """
    if M is None:
        M = int(x * math.sqrt(eps) + 30)
    n = math.sqrt(eps)
    m = np.arange(M + 1)
    j, jp = _bessel_j(x, M)
    jn, jnp = _bessel_j(n * x, M)
    h = special.hankel1(m, x)
    hp = special.h1vp(m, x)
    b = (jnp * j - n * jn * jp) / (n * jn * hp - jnp * h)
    base = alpha(m) * (-1j) ** m
    return _total_from_scattering(x, phi0, M, base * b * np.cos(m * phi0), base * b * np.sin(m * phi0))


def pec_te_coeffs(x: float, phi0: float = 0.0, M: int | None = None):
    """Homogeneous PEC cylinder, TE^z: E_phi = 0 on r = a, i.e. dHz/dr = 0,
    b_m = -J_m'(x) / H_m'(x)."""
    if M is None:
        M = int(x + 30)
    m = np.arange(M + 1)
    _, jp = _bessel_j(x, M)
    b = -jp / special.h1vp(m, x)
    base = alpha(m) * (-1j) ** m
    return _total_from_scattering(x, phi0, M, base * b * np.cos(m * phi0), base * b * np.sin(m * phi0))


def mdjc_surface_field(x: float, eps1: float, phi0: float, N: int, M: int | None = None):
    """Solve Eq. (matrix integral equation) for E_z^tot on phi_n = n dphi, n = 0..N-1.

    K(phi, phi') = sum_m (H_m'/H_m - 2 (k/k0) J_m'(ka)/J_m(ka)) sin m phi sin m phi'
                   + (alpha_m / 2) (H_m'/H_m) cos m phi cos m phi',
    Y(phi) = (2j / (k0 a)) sum_m alpha_m (-j)^m cos m(phi - phi0) / H_m(k0 a),
    k = k0 sqrt(eps1), dphi = pi / (N - 1).
    """
    if M is None:
        M = N - 1
    dphi = math.pi / (N - 1)
    phi = np.arange(N) * dphi
    m = np.arange(M + 1)
    hr, inv = _hankel_ratios(x, M)
    n = math.sqrt(eps1)
    jr = _bessel_j_ratio(n * x, M)
    a_sin = hr - 2.0 * n * jr
    a_cos = 0.5 * alpha(m) * hr
    sm = np.sin(np.outer(phi, m))
    cm = np.cos(np.outer(phi, m))
    K = (sm * a_sin) @ sm.T + (cm * a_cos) @ cm.T
    Y = (2j / x) * (np.cos(np.outer(phi, m) - m * phi0) @ (alpha(m) * (-1j) ** m * inv))
    E = np.linalg.solve(K * dphi, Y)
    return phi, E


def mdjc_coeffs(x: float, eps1: float, phi0: float, N: int, M: int | None = None, M_out: int | None = None):
    """C, S, C', S' (Eq. coefficients) of the metallo-dielectric Janus cylinder.

    Eq. (constants_Bm_Dm) with the rectangle rule of Eq. (discrete integral
    equation) gives B_m H_m + incident = C_m = (alpha_m / 2 pi) sum_n E_n cos(m phi_n) dphi
    and S_m = (1/pi) sum_n E_n sin(m phi_n) dphi; then
    C_m' = (H_m'/H_m) C_m + alpha_m (-j)^m cos(m phi0) (J_m' - J_m H_m'/H_m)
    with J_m' - J_m H_m'/H_m = -(2j / (pi x)) / H_m (Wronskian).
    """
    phi, E = mdjc_surface_field(x, eps1, phi0, N, M)
    if M_out is None:
        M_out = min(N - 1, int(3 * x + 60))
    dphi = phi[1] - phi[0]
    m = np.arange(M_out + 1)
    C = alpha(m) / (2 * math.pi) * (np.cos(np.outer(m, phi)) @ E) * dphi
    S = 1.0 / math.pi * (np.sin(np.outer(m, phi)) @ E) * dphi
    hr, inv = _hankel_ratios(x, M_out)
    w = -(2j / (math.pi * x)) * inv
    base = alpha(m) * (-1j) ** m
    Cp = hr * C + base * np.cos(m * phi0) * w
    Sp = hr * S + base * np.sin(m * phi0) * w
    return C, S, Cp, Sp


def forces_closed_form(C, S, Cp, Sp, x: float, phi0: float):
    """Eqs. (Fx), (Fy), (U), (V), (Torque): (F~x, F~y, M~z)."""
    R = np.real
    c = np.conj
    # the series is truncated at M; pad with zeros so every pair (m, m+1) and
    # triple (m-1, m, m+1) that touches a retained mode is summed
    C, S, Cp, Sp = (np.concatenate([np.asarray(v, dtype=complex), np.zeros(2, dtype=complex)]) for v in (C, S, Cp, Sp))
    M = len(C) - 1
    m = np.arange(M)  # m = 0..M-1 for the m, m+1 pairs
    U = (R(C[1] * c(C[0])) - R(S[1] * c(S[0])) + R(Cp[1] * c(Cp[0])) - R(Sp[1] * c(Sp[0])))
    U += np.sum(R(C[:-1] * c(C[1:])) + R(S[:-1] * c(S[1:])) + R(Cp[:-1] * c(Cp[1:])) + R(Sp[:-1] * c(Sp[1:])))
    U -= np.sum(m * (m + 1) * (R(C[:-1] * c(C[1:])) + R(S[:-1] * c(S[1:])))) / x ** 2
    k = np.arange(1, M)  # m = 1..M-1 for the m-1, m+1 triples
    inner = (Sp[0] * c(S[1]) - Cp[0] * c(C[1])) - np.sum(
        k * ((Cp[k - 1] - Cp[k + 1]) * c(C[k]) + (Sp[k - 1] - Sp[k + 1]) * c(S[k])))
    U -= R(inner) / x
    V = R(C[1] * c(S[0])) + R(C[0] * c(S[1])) + R(Cp[1] * c(Sp[0])) + R(Sp[1] * c(Cp[0]))
    V += np.sum(R(S[1:] * c(C[:-1])) - R(S[:-1] * c(C[1:])) + R(Cp[:-1] * c(Sp[1:])) - R(Sp[:-1] * c(Cp[1:])))
    V += np.sum(m * (m + 1) * (R(C[1:] * c(S[:-1])) - R(C[:-1] * c(S[1:])))) / x ** 2
    inner = (Cp[0] * c(S[1]) + Sp[0] * c(C[1])) + np.sum(
        k * ((Cp[k - 1] + Cp[k + 1]) * c(S[k]) - (Sp[k - 1] + Sp[k + 1]) * c(C[k])))
    V += R(inner) / x
    mm = np.arange(1, M + 1)
    T = np.sum(mm * R(Sp[1:] * c(C[1:]) - Cp[1:] * c(S[1:]))) / x
    fx = U * math.cos(phi0) + V * math.sin(phi0)
    fy = -U * math.sin(phi0) + V * math.cos(phi0)
    return fx, fy, T


def surface_fields(C, S, Cp, Sp, x: float, phi):
    """E_z, H_r, H_phi on r = a (Eq. total_field), with omega = k0, mu0 = 1, a = 1.

    Only quadratic forms of H enter the stress, so the sign convention of the
    curl equation does not matter.
    """
    m = np.arange(len(C))
    cm = np.cos(np.outer(phi, m))
    sm = np.sin(np.outer(phi, m))
    ez = cm @ C + sm @ S
    hr = (-1j / x) * ((-sm * m) @ C + (cm * m) @ S)
    hphi = 1j * (cm @ Cp + sm @ Sp)
    return ez, hr, hphi


def forces_quadrature(C, S, Cp, Sp, x: float, phi0: float, nq: int = 4096):
    """Eqs. (drag), (lift), (Torque) by the periodic trapezoid rule, normalised."""
    phi = 2 * math.pi * np.arange(nq) / nq
    ez, hr, hp = surface_fields(C, S, Cp, Sp, x, phi)
    nrm = -0.25 * np.abs(ez) ** 2 + 0.25 * (np.abs(hr) ** 2 - np.abs(hp) ** 2)
    sh = 0.5 * np.real(hp * np.conj(hr))
    cx = -math.cos(phi0) * np.cos(phi) - math.sin(phi0) * np.sin(phi)
    sx = -math.sin(phi0) * np.cos(phi) + math.cos(phi0) * np.sin(phi)
    cy = math.sin(phi0) * np.cos(phi) - math.cos(phi0) * np.sin(phi)
    sy = -math.cos(phi0) * np.cos(phi) - math.sin(phi0) * np.sin(phi)
    dphi = 2 * math.pi / nq
    a = 1.0
    fx = np.sum(nrm * cx + sh * sx) * a * dphi
    fy = np.sum(nrm * cy + sh * sy) * a * dphi
    tz = np.sum(sh) * a * a * dphi
    f0 = math.pi * a / 4.0
    return fx / f0, fy / f0, tz / (2 * f0 * a)


def forces_far_field(C, S, Cp, Sp, x: float, phi0: float, nq: int = 4096):
    """Drag and lift from the far field alone (momentum balance, lossless).

    B_m H_m = C_m - incident, so B_m = (C_m - inc_m)/H_m; far field
    E^S ~ sqrt(2/(pi k0 r)) exp(j(k0 r - pi/4)) T(phi), T = sum (-j)^m (B_m cos + D_m sin).
    For a lossless body the extinguished power equals the scattered power P,
    so F = P k_inc - (1/2) int (2/(pi k0)) |T|^2 r_hat dphi with
    P = (1/2) int (2/(pi k0)) |T|^2 dphi (eps0 = mu0 = c = 1).
    """
    M = len(C) - 1
    ic, is_, _, _ = incident_coeffs(x, phi0, M)
    _, inv = _hankel_ratios(x, M)
    B = (C - ic) * inv
    D = (S - is_) * inv
    phi = 2 * math.pi * np.arange(nq) / nq
    m = np.arange(M + 1)
    T = np.cos(np.outer(phi, m)) @ ((-1j) ** m * B) + np.sin(np.outer(phi, m)) @ ((-1j) ** m * D)
    dens = 0.5 * (2.0 / (math.pi * x)) * np.abs(T) ** 2   # per unit angle, k0 = x for a = 1
    dphi = 2 * math.pi / nq
    P = np.sum(dens) * dphi
    kin = math.pi + phi0
    Fb = np.array([P * math.cos(kin) - np.sum(dens * np.cos(phi)) * dphi,
                   P * math.sin(kin) - np.sum(dens * np.sin(phi)) * dphi])
    ex = np.array([math.cos(kin), math.sin(kin)])
    ey = np.array([math.cos(kin + math.pi / 2), math.sin(kin + math.pi / 2)])
    f0 = math.pi / 4.0
    return float(Fb @ ex) / f0, float(Fb @ ey) / f0


def mdjc_forces(x: float, eps1: float, phi0: float, N: int):
    C, S, Cp, Sp = mdjc_coeffs(x, eps1, phi0, N)
    return forces_closed_form(C, S, Cp, Sp, x, phi0)


def mdjc_forces_extrapolated(x: float, eps1: float, phi0: float, N: int = 1025, p: float | None = None):
    """Richardson extrapolation over N, 2N-1, 4N-3 (dphi halves each time).

    With the fitted order p (if None, taken from the three drag values when
    they are monotone, else 4/3), Q_inf = Q_3 + (Q_3 - Q_2) / (2^p - 1).
    """
    q1 = np.array(mdjc_forces(x, eps1, phi0, N))
    q2 = np.array(mdjc_forces(x, eps1, phi0, 2 * N - 1))
    q3 = np.array(mdjc_forces(x, eps1, phi0, 4 * N - 3))
    if p is None:
        d1, d2 = q2[0] - q1[0], q3[0] - q2[0]
        p = math.log2(d1 / d2) if d1 * d2 > 0 and abs(d2) > 1e-14 else 4.0 / 3.0
        if not (0.5 < p < 3.0):
            p = 4.0 / 3.0
    return tuple(q3 + (q3 - q2) / (2 ** p - 1)), p, (q1, q2, q3)


# ----------------------------------------------------------------------------
# Far field (Sec. II.A): scattering intensity |S(phi)|^2 = k0 r |E^S|^2 / |E^I|^2
# ----------------------------------------------------------------------------


def scattering_coeffs(C, S, x: float, phi0: float):
    """B_m, D_m of Eq. (scattered field) from the total-field coefficients on
    r = a: B_m H_m(x) = C_m - incident_m (and likewise D_m with S_m)."""
    M = len(C) - 1
    ic, is_, _, _ = incident_coeffs(x, phi0, M)
    _, inv = _hankel_ratios(x, M)
    return (np.asarray(C) - ic) * inv, (np.asarray(S) - is_) * inv


def far_intensity(B, D, phi):
    """|S(phi)|^2 at body angles phi for a unit incident amplitude.

    H_m(z) ~ sqrt(2 / (pi z)) exp(j (z - m pi / 2 - pi / 4)) for large z, so
    k0 r |E^S|^2 -> (2 / pi) |sum_m (-j)^m (B_m cos m phi + D_m sin m phi)|^2.
    """
    m = np.arange(len(B))
    phi = np.atleast_1d(np.asarray(phi, dtype=float))
    T = np.cos(np.outer(phi, m)) @ ((-1j) ** m * B) + np.sin(np.outer(phi, m)) @ ((-1j) ** m * D)
    return 2.0 / math.pi * np.abs(T) ** 2


def scattered_near_field(B, D, k0: float, R: float, phi):
    """E_z^S, H_x^S, H_y^S at r = R, body angles phi (Cartesian components in
    the body frame), time factor exp(-j omega t), eps0 = mu0 = 1, so that
    curl E = j k0 H: H_x = (dE_z/dy) / (j k0), H_y = -(dE_z/dx) / (j k0)."""
    m = np.arange(len(B))
    z = k0 * R
    h = special.hankel1(m, z)
    hp = special.h1vp(m, z)
    phi = np.asarray(phi, dtype=float)
    cm, sm = np.cos(np.outer(phi, m)), np.sin(np.outer(phi, m))
    ez = cm @ (B * h) + sm @ (D * h)
    d_r = k0 * (cm @ (B * hp) + sm @ (D * hp))
    d_phi = (-sm * m) @ (B * h) + (cm * m) @ (D * h)
    dx = np.cos(phi) * d_r - np.sin(phi) / R * d_phi
    dy = np.sin(phi) * d_r + np.cos(phi) / R * d_phi
    return ez, dy / (1j * k0), -dx / (1j * k0)
