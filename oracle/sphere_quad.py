"""Surface integrals over spheres by product quadrature (oracle side).

Test infrastructure (see the package docstring).

Sec. 3.5 evaluates the integrals that carry a Dirac delta of the distance,
int f(r') delta(|r' - r| - R) dr', by changing to spherical coordinates
about r: the delta removes the radial integral and leaves R^2 times the
integral of f over the sphere of radius R, written in the azimuth theta in
[0, 2 pi) and the polar angle phi in [0, pi] with the Jacobian sin(phi),
and approximated by a k-by-k product rule in (theta, phi).  Integrand points
off the grid are interpolated; the paper leaves open both the 1D rules and
the interpolation, and extends the integrand by zero outside the domain.
The readings taken here:

  * theta: k equispaced points theta_i = 2 pi i / k, weight 2 pi / k each
    (the trapezoidal rule of a periodic integrand);
  * phi: k Gauss-Legendre points mapped from [-1, 1] onto [0, pi], weights
    scaled by pi / 2, with sin(phi_j) in the integrand as in the paper's sum;
  * the integrand between grid points: trilinear interpolation of the
    grid values (exact for affine fields), or, with cubic=True, the
    tricubic interpolant through the 4 x 4 x 4 grid points around the node
    (Lagrange cubics on the offsets -1, 0, 1, 2 of each axis: exact for
    polynomials of degree 3 in each coordinate);
  * outside the grid: periodic images (the periodic box of the rest of the
    evaluation), or zero (the paper's zero extension; `aperiodic=True`).

Alongside the scalar integral the vector one is formed, R^2 times the
sphere integral of f(r + R n) n, which is the FMT vector weighted density
n_2v of one species in this code's correlation convention (weight x/|x| at
the displacement x = r' - r).  So for the FMT weights of Sec. 2.3.1 with
R_i = d_i / 2: n_2 = sum_i I_i, n_1 = sum_i I_i / (4 pi R_i),
n_0 = sum_i I_i / (4 pi R_i^2), n_2v = sum_i I_v,i, n_1v = sum_i I_v,i / (4 pi R_i).

The smoothed-delta alternative that the paper argues against
(delta replaced by a Gaussian of width alpha, then an ordinary volume rule)
is `shell_integral_gaussian_delta`, kept for the accuracy comparison.
"""
import math

import numpy as np


def sphere_rule(k):
    """The k-by-k product rule: (theta [k], w_theta [k], phi [k], w_phi [k])."""
    if k < 1:
        raise ValueError("order must be >= 1")
    theta = 2.0 * math.pi * np.arange(k) / k
    w_theta = np.full(k, 2.0 * math.pi / k)
    x, w = np.polynomial.legendre.leggauss(k)
    phi = 0.5 * math.pi * (x + 1.0)
    w_phi = 0.5 * math.pi * w
    return theta, w_theta, phi, w_phi


def _shifted(f, base, aperiodic):
    """f at every grid point r + base (integer 3-vector), periodic or zero outside."""
    if not aperiodic:
        return np.roll(f, shift=(-base[0], -base[1], -base[2]), axis=(0, 1, 2))
    out = np.zeros_like(f)
    src = []
    dst = []
    for a in range(3):
        n = f.shape[a]
        lo = max(0, -base[a])
        hi = min(n, n - base[a])
        if hi <= lo:
            return out
        dst.append(slice(lo, hi))
        src.append(slice(lo + base[a], hi + base[a]))
    out[tuple(dst)] = f[tuple(src)]
    return out


def axis_weights(t, cubic=False):
    """Interpolation offsets along one axis and their weights at fraction t
    (the node lies at base + t, base = floor): linear, the two points
    (0, 1) with (1 - t, t); cubic, the four points (-1, 0, 1, 2) with the
    Lagrange cubics through them evaluated at t.  t may be an array."""
    t = np.asarray(t, dtype=np.float64)
    if not cubic:
        return (0, 1), (1.0 - t, t)
    return (-1, 0, 1, 2), (-t * (t - 1.0) * (t - 2.0) / 6.0,
                           (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0,
                           -(t + 1.0) * t * (t - 2.0) / 2.0,
                           (t + 1.0) * t * (t - 1.0) / 6.0)


def interpolate_shifted(f, p, aperiodic=False, cubic=False):
    """Interpolant of the grid function f at r + p for every grid point r.

    p is a displacement in grid units (3 floats).  Trilinear: the eight
    corners of the cell that holds r + p, weighted by the products of the
    fractional distances (the textbook formula); cubic: the products of the
    per-axis Lagrange weights of `axis_weights` over 4 x 4 x 4 points.
    """
    p = np.asarray(p, dtype=np.float64)
    base = np.floor(p).astype(np.int64)
    t = p - base
    offs = [axis_weights(t[a], cubic) for a in range(3)]
    out = np.zeros_like(f)
    for ox, wx in zip(*offs[0]):
        for oy, wy in zip(*offs[1]):
            for oz, wz in zip(*offs[2]):
                wgt = float(wx * wy * wz)
                if wgt == 0.0:
                    continue
                out += wgt * _shifted(f, base + np.array([ox, oy, oz]), aperiodic)
    return out


def shell_integrals(f, R, h, k, aperiodic=False, cubic=False):
    """Sec. 3.5 product quadrature of one field on the sphere of radius R about every grid point.

    f: [nx, ny, nz] grid values (z fastest); R, h in the same length unit.
    Returns (I [nx,ny,nz], Iv [3, nx,ny,nz]):
      I(r)  ~ sum_i sum_j f(r + R n_ij) R^2 sin(phi_j) w_i w~_j
      Iv(r) ~ the same sum with f(r + R n_ij) n_ij in place of f(r + R n_ij),
    n_ij = (cos theta_i sin phi_j, sin theta_i sin phi_j, cos phi_j).
    """
    f = np.asarray(f, dtype=np.float64)
    theta, w_theta, phi, w_phi = sphere_rule(k)
    scalar = np.zeros_like(f)
    vector = np.zeros((3,) + f.shape)
    for i in range(k):
        for j in range(k):
            n = np.array([math.cos(theta[i]) * math.sin(phi[j]),
                          math.sin(theta[i]) * math.sin(phi[j]),
                          math.cos(phi[j])])
            weight = R * R * math.sin(phi[j]) * w_theta[i] * w_phi[j]
            g = interpolate_shifted(f, (R / h) * n, aperiodic, cubic)
            scalar += weight * g
            for a in range(3):
                vector[a] += (weight * n[a]) * g
    return scalar, vector


def shell_integrals_at(f, R, h, k, points, aperiodic=False, cubic=False):
    """The same sums as `shell_integrals`, at chosen grid points only.

    points: [P, 3] integer grid indices.  Each node position r + R n / h is
    interpolated on its own (floor, fractions, eight or 64 points), for
    sampled checks on grids too large for the whole-grid form.
    Returns (I [P], Iv [3, P]).
    """
    f = np.asarray(f, dtype=np.float64)
    pts = np.asarray(points, dtype=np.int64)
    shape = np.array(f.shape)
    theta, w_theta, phi, w_phi = sphere_rule(k)
    scalar = np.zeros(len(pts))
    vector = np.zeros((3, len(pts)))
    for i in range(k):
        for j in range(k):
            n = np.array([math.cos(theta[i]) * math.sin(phi[j]),
                          math.sin(theta[i]) * math.sin(phi[j]),
                          math.cos(phi[j])])
            weight = R * R * math.sin(phi[j]) * w_theta[i] * w_phi[j]
            pos = pts + (R / h) * n
            base = np.floor(pos).astype(np.int64)
            t = pos - base
            g = np.zeros(len(pts))
            offs = [axis_weights(t[:, a], cubic) for a in range(3)]
            for cx, wx in zip(*offs[0]):
                for cy, wy in zip(*offs[1]):
                    for cz, wz in zip(*offs[2]):
                        c = np.array([cx, cy, cz])
                        wgt = wx * wy * wz
                        idx = base + c
                        if aperiodic:
                            inside = np.all((idx >= 0) & (idx < shape), axis=1)
                            idx = np.clip(idx, 0, shape - 1)
                            val = np.where(inside, f[idx[:, 0], idx[:, 1], idx[:, 2]], 0.0)
                        else:
                            idx = np.mod(idx, shape)
                            val = f[idx[:, 0], idx[:, 1], idx[:, 2]]
                        g += wgt * val
            scalar += weight * g
            for a in range(3):
                vector[a] += (weight * n[a]) * g
    return scalar, vector


def shell_weighted_densities(rho, radii, h, k, aperiodic=False, cubic=False):
    """n0, n1, n2, n1v, n2v of Sec. 2.3.1 from the sphere quadrature (n3 is a volume integral, not here).

    rho: [S, nx, ny, nz]; radii: S sphere radii R_i = d_i / 2.
    Returns a dict of arrays (vectors [3, ...]).
    """
    rho = np.asarray(rho, dtype=np.float64)
    shape = rho.shape[1:]
    acc = {"n0": np.zeros(shape), "n1": np.zeros(shape), "n2": np.zeros(shape),
           "n1v": np.zeros((3,) + shape), "n2v": np.zeros((3,) + shape)}
    for i, R in enumerate(radii):
        I, Iv = shell_integrals(rho[i], R, h, k, aperiodic, cubic)
        acc["n2"] += I
        acc["n1"] += I / (4.0 * math.pi * R)
        acc["n0"] += I / (4.0 * math.pi * R * R)
        acc["n2v"] += Iv
        acc["n1v"] += Iv / (4.0 * math.pi * R)
    return acc


def gaussian_bump_shell(d, R, s, amplitude=1.0):
    """Exact sphere integrals of amplitude * exp(-|x - c|^2 / (2 s^2)) at distance d from c.

    Returns (I, Iv_radial): I = int f(r') delta(|r' - r| - R) dr', and the
    component of the vector integral along (r - c)/d.  Reduced by hand to one
    polar integral of exp(-(d^2 + R^2 + 2 d R u) / (2 s^2)) (times u for the
    vector), which is elementary.
    """
    d = np.asarray(d, dtype=np.float64)
    A = (d * d + R * R) / (2.0 * s * s)
    B = d * R / (s * s)
    small = B < 1e-6
    Bs = np.where(small, 1.0, B)
    # int_{-1}^{1} exp(-B u) du = 2 sinh(B) / B ;  int u exp(-B u) du = 2 sinh(B)/B^2 - 2 cosh(B)/B
    # (written with exponentials of -A +- B to stay finite for large B)
    e_m = np.exp(-A + Bs)
    e_p = np.exp(-A - Bs)
    s0 = np.where(small, 2.0 * np.exp(-A), (e_m - e_p) / Bs)
    s1 = np.where(small, -2.0 * B / 3.0 * np.exp(-A),
                  (e_m - e_p) / (Bs * Bs) - (e_m + e_p) / Bs)
    return amplitude * 2.0 * math.pi * R * R * s0, amplitude * 2.0 * math.pi * R * R * s1


def shell_integral_gaussian_delta(f, R, h, alpha, aperiodic=False):
    """The smoothed-delta route: delta(|x| - R) ~ exp(-(|x| - R)^2 / alpha^2) / (alpha sqrt(pi)),
    then the grid (rectangle) rule over all displacements with |x| <= R + 8 alpha.

    Returns I [nx, ny, nz] (scalar integral only).
    """
    f = np.asarray(f, dtype=np.float64)
    reach = int(math.ceil((R + 8.0 * alpha) / h))
    out = np.zeros_like(f)
    for dx in range(-reach, reach + 1):
        for dy in range(-reach, reach + 1):
            for dz in range(-reach, reach + 1):
                r = h * math.sqrt(dx * dx + dy * dy + dz * dz)
                if r > R + 8.0 * alpha:
                    continue
                w = math.exp(-((r - R) / alpha) ** 2) / (alpha * math.sqrt(math.pi)) * h ** 3
                out += w * _shifted(f, np.array([dx, dy, dz]), aperiodic)
    return out
