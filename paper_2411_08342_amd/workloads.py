"""Seeded synthetic inputs: surfaces, targets and near lists.

This module only generates inputs (geometry, collocation nodes, boundary edge
samples, targets, near lists, densities).  It contains none of the quadrature
method's arithmetic and is shared by the tests, the benchmark and the oracle
tests as the single source of inputs.

Surfaces are unions of quadrilateral patches, each the image of [-1, 1]^2
under an analytic map.  Every patch carries
* a q x q tensor Gauss-Legendre grid of nodes (node index a*q + b: v = t_a, u = t_b),
  exact unit outward normals and smooth-rule weights w = w_a w_b |r_u x r_v|;
* four edges, counter-clockwise about the outward normal
  (v=-1: u=t; u=1: v=t; v=1: u=-t; u=-1: v=-t), each sampled at the ptilde
  Gauss-Legendre parameters t in increasing order.  Neighbouring patches share
  their edge curves, so the samples of a shared edge coincide.
Tangent derivatives come from complex-step differentiation of the analytic maps.
"""
import math

import numpy as np

SEED_BASE = 20241113
_CS_H = 1e-30


def gl(n):
    return np.polynomial.legendre.leggauss(n)


# ----------------------------------------------------------------------------
# analytic maps (written with complex-step safe operations only)
# ----------------------------------------------------------------------------

def _face_dir(f, a, b):
    """Equiangular cubed-sphere chart f: (a, b) = (tan xi, tan eta) -> unnormalised direction,
    oriented so that d/da x d/db points outward."""
    one = np.ones_like(a)
    if f == 0:
        return one, a, b
    if f == 1:
        return -one, b, a
    if f == 2:
        return -a, one, b
    if f == 3:
        return a, -one, b
    if f == 4:
        return -b, a, one
    return b, a, -one


def cubed_sphere_dir(f, xi, eta):
    x, y, z = _face_dir(f, np.tan(xi), np.tan(eta))
    n = np.sqrt(x * x + y * y + z * z)
    return x / n, y / n, z / n


def real_sph_harm_unit(L, x, y, z):
    """Orthonormal real spherical harmonics Y_lm(x, y, z), |(x,y,z)| = 1, l <= L, as a dict
    {(l, m): values}, m < 0 the sine family.  Written with polynomial recurrences only."""
    C = [np.ones_like(x)]
    Sn = [np.zeros_like(x)]
    for m in range(1, L + 1):
        C.append(x * C[m - 1] - y * Sn[m - 1])
        Sn.append(x * Sn[m - 1] + y * C[m - 1])
    out = {}
    for m in range(0, L + 1):
        # Pbar_l^m(z) = P_l^m(z) / (1 - z^2)^{m/2}: polynomial in z
        pmm = math.prod(range(1, 2 * m, 2)) if m > 0 else 1.0
        pb = {m: pmm * np.ones_like(z)}
        if m + 1 <= L:
            pb[m + 1] = (2 * m + 1) * z * pb[m]
        for l in range(m + 1, L):
            pb[l + 1] = ((2 * l + 1) * z * pb[l] - (l + m) * pb[l - 1]) / (l - m + 1)
        for l in range(m, L + 1):
            nrm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
            if m == 0:
                out[(l, 0)] = nrm * pb[l]
            else:
                out[(l, m)] = math.sqrt(2) * nrm * pb[l] * C[m]
                out[(l, -m)] = math.sqrt(2) * nrm * pb[l] * Sn[m]
    return out


def star_radius(x, y, z):
    """1 + 0.2 Re Y_4^3 + 0.1 Re Y_2^1 on the unit sphere, with the paper's normalisation of
    Y_l^m (no 1/sqrt(4 pi), no Condon-Shortley phase)."""
    c43 = 3.0 * 105.0 / math.sqrt(math.factorial(7))      # sqrt(9) sqrt(1/7!) * 105
    c21 = math.sqrt(5.0) * 3.0 / math.sqrt(6.0)            # sqrt(5) sqrt(1/3!) * 3
    return 1.0 + 0.2 * c43 * z * (x ** 3 - 3 * x * y * y) + 0.1 * c21 * z * x


class PatchMap:
    """r(u, v) on [-1, 1]^2 for one patch."""

    def __init__(self, fn):
        self.fn = fn

    def __call__(self, u, v):
        return self.fn(u, v)

    def derivs(self, u, v):
        u = np.asarray(u, dtype=np.float64)
        v = np.asarray(v, dtype=np.float64)
        ru = np.stack(self.fn(u + 1j * _CS_H, v + 0j), axis=-1).imag / _CS_H
        rv = np.stack(self.fn(u + 0j, v + 1j * _CS_H), axis=-1).imag / _CS_H
        r = np.stack(self.fn(u, v), axis=-1).real
        return r, ru, rv


def cubed_sphere_patches(n, radial=None, scale=(1.0, 1.0, 1.0), rot=None, center=(0, 0, 0)):
    """6 n^2 patches of a (deformed, scaled, rotated, shifted) cubed sphere."""
    edges = np.linspace(-math.pi / 4, math.pi / 4, n + 1)
    rot = np.eye(3) if rot is None else np.asarray(rot)
    maps = []
    for f in range(6):
        for i in range(n):
            for j in range(n):
                x0, x1 = edges[j], edges[j + 1]
                y0, y1 = edges[i], edges[i + 1]

                def fn(u, v, f=f, x0=x0, x1=x1, y0=y0, y1=y1):
                    xi = 0.5 * (x0 + x1) + 0.5 * (x1 - x0) * u
                    eta = 0.5 * (y0 + y1) + 0.5 * (y1 - y0) * v
                    dx, dy, dz = cubed_sphere_dir(f, xi, eta)
                    rr = 1.0 if radial is None else radial(dx, dy, dz)
                    p = (scale[0] * rr * dx, scale[1] * rr * dy, scale[2] * rr * dz)
                    return tuple(rot[a, 0] * p[0] + rot[a, 1] * p[1] + rot[a, 2] * p[2] + center[a]
                                 for a in range(3))
                maps.append(PatchMap(fn))
    return maps


def torus_patches(nt, nphi, R=1.0, r=0.35, center=(0, 0, 0)):
    maps = []
    for i in range(nt):
        for j in range(nphi):
            t0, t1 = 2 * math.pi * i / nt, 2 * math.pi * (i + 1) / nt
            p0, p1 = 2 * math.pi * j / nphi, 2 * math.pi * (j + 1) / nphi

            def fn(u, v, t0=t0, t1=t1, p0=p0, p1=p1):
                # u along phi (toroidal), v along theta (poloidal): r_u x r_v outward
                ph = 0.5 * (p0 + p1) + 0.5 * (p1 - p0) * u
                th = 0.5 * (t0 + t1) + 0.5 * (t1 - t0) * v
                rho = R + r * np.cos(th)
                return (rho * np.cos(ph) + center[0], rho * np.sin(ph) + center[1],
                        r * np.sin(th) + center[2])
            maps.append(PatchMap(fn))
    return maps


# ----------------------------------------------------------------------------
# discretisation
# ----------------------------------------------------------------------------

def _edge_params(t):
    one = np.ones_like(t)
    return [(t, -one), (one, t), (-t, one), (-one, -t)]


def discretize(maps, orders, ptilde_factor=2):
    """SoA surface description from patch maps and per-patch orders q."""
    orders = np.asarray(orders, dtype=np.int32)
    P = len(maps)
    node_off = np.zeros(P + 1, dtype=np.int64)
    node_off[1:] = np.cumsum(orders.astype(np.int64) ** 2)
    pt = (ptilde_factor * orders).astype(np.int64)
    edge_off = np.zeros(P + 1, dtype=np.int64)
    edge_off[1:] = np.cumsum(4 * pt)
    N, E = int(node_off[-1]), int(edge_off[-1])
    xyz = np.zeros((3, N))
    nrm = np.zeros((3, N))
    wt = np.zeros(N)
    exyz = np.zeros((3, E))
    corners = np.zeros((P, 4, 3))
    rules = {}
    for P_, m in enumerate(maps):
        q = int(orders[P_])
        if q not in rules:
            rules[q] = gl(q)
        t, w = rules[q]
        V, U = np.meshgrid(t, t, indexing="ij")
        r, ru, rv = m.derivs(U.reshape(-1), V.reshape(-1))
        nv = np.cross(ru, rv)
        J = np.linalg.norm(nv, axis=1)
        a, b = node_off[P_], node_off[P_ + 1]
        xyz[:, a:b] = r.T
        nrm[:, a:b] = (nv / J[:, None]).T
        wt[a:b] = np.outer(w, w).reshape(-1) * J
        n_e = int(pt[P_])
        if n_e not in rules:
            rules[n_e] = gl(n_e)
        te, _ = rules[n_e]
        ea = edge_off[P_]
        for e, (uu, vv) in enumerate(_edge_params(te)):
            pts = np.stack(m(uu, vv), axis=-1).real
            exyz[:, ea + e * n_e: ea + (e + 1) * n_e] = pts.T
        cu = np.array([-1.0, 1.0, 1.0, -1.0])
        cv = np.array([-1.0, -1.0, 1.0, 1.0])
        corners[P_] = np.stack(m(cu, cv), axis=-1).real
    return dict(npatch=P, order=orders, node_off=node_off, node_xyz=xyz, node_nrm=nrm,
                node_wt=wt, edge_off=edge_off, edge_xyz=exyz, corners=corners, maps=maps)


def patch_center_diam(surface):
    c = surface["corners"]
    ctr = c.mean(axis=1)
    diam = np.max(np.linalg.norm(c[:, :, None, :] - c[:, None, :, :], axis=-1), axis=(1, 2))
    return ctr, diam


def node_targets(surface):
    P = surface["npatch"]
    off = surface["node_off"]
    sp = np.repeat(np.arange(P, dtype=np.int32), np.diff(off))
    sn = (np.arange(off[-1]) - off[sp]).astype(np.int32)
    return surface["node_xyz"].copy(), surface["node_nrm"].copy(), sp, sn


def offsurface_targets(surface, rng, count_per_patch=None, total=None, rel_dist=None,
                       abs_dist=None):
    """Targets = foot point (uniform parameter point of a patch) + offset along the foot
    normal, random side.  Offsets log-uniform in rel_dist * D_P or abs_dist."""
    P = surface["npatch"]
    _, diam = patch_center_diam(surface)
    if count_per_patch is not None:
        patches = np.repeat(np.arange(P), count_per_patch)
    else:
        patches = rng.integers(0, P, size=total)
    n = len(patches)
    u = rng.uniform(-1, 1, n)
    v = rng.uniform(-1, 1, n)
    lo, hi = rel_dist if rel_dist is not None else abs_dist
    dist = np.exp(rng.uniform(math.log(lo), math.log(hi), n))
    if rel_dist is not None:
        dist = dist * diam[patches]
    side = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    xyz = np.zeros((3, n))
    nrm = np.zeros((3, n))
    for P_ in np.unique(patches):
        sel = np.nonzero(patches == P_)[0]
        r, ru, rv = surface["maps"][P_].derivs(u[sel], v[sel])
        nv = np.cross(ru, rv)
        nv /= np.linalg.norm(nv, axis=1)[:, None]
        xyz[:, sel] = (r + (side[sel] * dist[sel])[:, None] * nv).T
        nrm[:, sel] = nv.T
    return xyz, nrm


def near_lists(surface, xyz, eta):
    """CSR near list: patch P is near target x iff |x - c_P| < eta * D_P
    (c_P: mean of the corners, D_P: largest corner distance)."""
    from scipy.spatial import cKDTree
    ctr, diam = patch_center_diam(surface)
    tree = cKDTree(xyz.T)
    rows, cols = [], []
    for P_ in range(surface["npatch"]):
        hits = tree.query_ball_point(ctr[P_], eta * diam[P_])
        if hits:
            rows.append(np.asarray(hits, dtype=np.int64))
            cols.append(np.full(len(hits), P_, dtype=np.int32))
    T = xyz.shape[1]
    if rows:
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
    else:
        rows = np.zeros(0, dtype=np.int64)
        cols = np.zeros(0, dtype=np.int32)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    ptr = np.zeros(T + 1, dtype=np.int64)
    np.add.at(ptr, rows + 1, 1)
    ptr = np.cumsum(ptr)
    return ptr, cols.astype(np.int32)


def make_targets(surface, xyz, nrm, self_patch, self_node, eta):
    ptr, near = near_lists(surface, xyz, eta)
    return dict(ntarget=xyz.shape[1], xyz=np.ascontiguousarray(xyz),
                nrm=np.ascontiguousarray(nrm),
                self_patch=np.asarray(self_patch, dtype=np.int32),
                self_node=np.asarray(self_node, dtype=np.int32), near_ptr=ptr, near_patch=near)


def merge_surfaces(surfs):
    """Concatenate surface descriptions (patch, node and edge indices shifted)."""
    out = dict(npatch=sum(s["npatch"] for s in surfs))
    out["order"] = np.concatenate([s["order"] for s in surfs])
    for off_key in ("node_off", "edge_off"):
        parts, base = [np.zeros(1, dtype=np.int64)], 0
        for s in surfs:
            parts.append(s[off_key][1:] + base)
            base += s[off_key][-1]
        out[off_key] = np.concatenate(parts)
    for k in ("node_xyz", "node_nrm", "edge_xyz"):
        out[k] = np.concatenate([s[k] for s in surfs], axis=1)
    out["node_wt"] = np.concatenate([s["node_wt"] for s in surfs])
    out["corners"] = np.concatenate([s["corners"] for s in surfs])
    out["maps"] = sum((s["maps"] for s in surfs), [])
    return out


# ----------------------------------------------------------------------------
# the workloads of the evaluation (synthetic stand-ins of the paper's tests)
# ----------------------------------------------------------------------------

def sphere_q6():
    """Unit sphere, 6 cubed-sphere patches, q = 6; density Re Y_3^2; 216 node targets and
    200 off-surface targets (100 inside, 100 outside) at log-uniform distances [1e-4, 1e-1]."""
    rng = np.random.default_rng(SEED_BASE + 1)
    surf = discretize(cubed_sphere_patches(1), np.full(6, 6))
    x, n, sp, sn = node_targets(surf)
    m = 200
    d = rng.normal(size=(3, m))
    d /= np.linalg.norm(d, axis=0)
    dist = np.exp(rng.uniform(math.log(1e-4), math.log(1e-1), m))
    rad = np.where(np.arange(m) < m // 2, 1.0 - dist, 1.0 + dist)
    xo = d * rad
    xyz = np.concatenate([x, xo], axis=1)
    nrm = np.concatenate([n, d], axis=1)
    sp = np.concatenate([sp, np.full(m, -1, np.int32)])
    sn = np.concatenate([sn, np.full(m, -1, np.int32)])
    tg = make_targets(surf, xyz, nrm, sp, sn, eta=1.0)
    X, Y, Z = surf["node_xyz"]
    dens = math.sqrt(7.0 / 120.0) * 15.0 * Z * (X * X - Y * Y)
    return surf, tg, dens


def _random_density(rng, xyz, L=6):
    r = np.linalg.norm(xyz, axis=0)
    Y = real_sph_harm_unit(L, *(xyz / r))
    return sum(rng.normal() * Y[k] for k in sorted(Y))


def star(n=16, q=8):
    """Star-shaped surface r = 1 + 0.2 Re Y_4^3 + 0.1 Re Y_2^1, 6 n^2 patches of order q;
    targets all nodes, near radius 1.5 patch diameters."""
    rng = np.random.default_rng(SEED_BASE + 2)
    surf = discretize(cubed_sphere_patches(n, radial=star_radius), np.full(6 * n * n, q))
    x, nn, sp, sn = node_targets(surf)
    tg = make_targets(surf, x, nn, sp, sn, eta=1.5)
    return surf, tg, _random_density(rng, surf["node_xyz"])


def _random_rotation(rng):
    Qm, Rm = np.linalg.qr(rng.normal(size=(3, 3)))
    Qm = Qm * np.sign(np.diag(Rm))[None, :]
    if np.linalg.det(Qm) < 0:
        Qm[:, 0] = -Qm[:, 0]
    return Qm


def ellipsoids_mixed_orders(n_ell=12, nmin=4, nmax=16, orders=(4, 6, 8, 10), mean_targets=150):
    """12 ellipsoids (semi-axes U[0.5, 2]), seeded rotations, non-overlapping bounding
    spheres; 6 n^2 patches each with n ~ U{nmin..nmax}; per-patch order from `orders`;
    Poisson(mean_targets) off-surface targets per patch at log-U[1e-5, 0.5] D_P."""
    rng = np.random.default_rng(SEED_BASE + 3)
    surfs, centers, radii = [], [], []
    for e in range(n_ell):
        ax = rng.uniform(0.5, 2.0, 3)
        rb = ax.max()
        for _ in range(10000):
            c = rng.uniform(-8, 8, 3)
            if all(np.linalg.norm(c - c2) > rb + r2 + 0.1 for c2, r2 in zip(centers, radii)):
                break
        centers.append(c)
        radii.append(rb)
        n = int(rng.integers(nmin, nmax + 1))
        maps = cubed_sphere_patches(n, scale=tuple(ax), rot=_random_rotation(rng), center=tuple(c))
        ords = rng.choice(np.asarray(orders), size=len(maps))
        surfs.append(discretize(maps, ords))
    surf = merge_surfaces(surfs)
    counts = rng.poisson(mean_targets, surf["npatch"])
    xyz, nrm = offsurface_targets(surf, rng, count_per_patch=counts, rel_dist=(1e-5, 0.5))
    T = xyz.shape[1]
    tg = make_targets(surf, xyz, nrm, np.full(T, -1), np.full(T, -1), eta=1.0)
    return surf, tg, None


def star_torus(n=16, q=8, nt=32, nphi=64):
    """The star surface plus a torus (R = 1, r = 0.35, nt x nphi patches, order q) placed
    beside it; targets all nodes of both surfaces."""
    s1 = discretize(cubed_sphere_patches(n, radial=star_radius), np.full(6 * n * n, q))
    s2 = discretize(torus_patches(nt, nphi, center=(3.0, 0.0, 0.0)), np.full(nt * nphi, q))
    surf = merge_surfaces([s1, s2])
    x, nn, sp, sn = node_targets(surf)
    tg = make_targets(surf, x, nn, sp, sn, eta=1.5)
    return surf, tg, None


def forty_spheres(cloud=200_000, spheres=40, lattice=(4, 5, 2), spacing=2.3,
            ns=(9,) * 3 + (10,) * 33 + (11,) + (12,) * 3, q=8):
    """40 deformed spheres r = 1 + sum_{l<=5} a_lm Y_lm (orthonormal real basis, a ~ N(0, 0.03^2))
    on a lattice with spacing 2.3; sub-grid sizes n as listed (24,576 patches, order 8); targets
    all nodes plus an off-surface cloud at log-U[1e-6, 0.3] absolute distance."""
    rng = np.random.default_rng(SEED_BASE + 5)
    surfs = []
    k = 0
    for ix in range(lattice[0]):
        for iy in range(lattice[1]):
            for iz in range(lattice[2]):
                if k >= spheres:
                    break
                coeff = {(l, m): rng.normal(0, 0.03) for l in range(0, 6) for m in range(-l, l + 1)}

                def radial(x, y, z, coeff=coeff):
                    Y = real_sph_harm_unit(5, x, y, z)
                    return 1.0 + sum(c * Y[key] for key, c in coeff.items())
                maps = cubed_sphere_patches(ns[k], radial=radial,
                                            center=(ix * spacing, iy * spacing, iz * spacing))
                surfs.append(discretize(maps, np.full(len(maps), q)))
                k += 1
    surf = merge_surfaces(surfs)
    x, nn, sp, sn = node_targets(surf)
    xo, no = offsurface_targets(surf, rng, total=cloud, abs_dist=(1e-6, 0.3))
    xyz = np.concatenate([x, xo], axis=1)
    nrm = np.concatenate([nn, no], axis=1)
    sp = np.concatenate([sp, np.full(xo.shape[1], -1, np.int32)])
    sn = np.concatenate([sn, np.full(xo.shape[1], -1, np.int32)])
    tg = make_targets(surf, xyz, nrm, sp, sn, eta=1.0)
    return surf, tg, None


def learned_guess_training(seed=SEED_BASE + 40, n=10, q=8, nt=20, nphi=40, per_patch=12):
    """Seeded geometry for the learned Newton guess's training samples, kept apart from the
    evaluation surfaces: a deformed sphere r = 1 + sum_{l<=5} a_lm Y_lm (a ~ N(0, 0.06^2))
    and a torus (R = 1.1, r = 0.4) beside it, order q; targets all nodes plus per_patch
    off-surface points per patch at distances log-U[1e-4, 0.5] patch diameters; near list
    1.5 patch diameters."""
    rng = np.random.default_rng(seed)
    coeff = {(l, m): rng.normal(0, 0.06) for l in range(0, 6) for m in range(-l, l + 1)}

    def radial(x, y, z):
        Y = real_sph_harm_unit(5, x, y, z)
        return 1.0 + sum(c * Y[key] for key, c in coeff.items())
    s1 = discretize(cubed_sphere_patches(n, radial=radial), np.full(6 * n * n, q))
    s2 = discretize(torus_patches(nt, nphi, R=1.1, r=0.4, center=(3.2, 0.0, 0.0)),
                    np.full(nt * nphi, q))
    surf = merge_surfaces([s1, s2])
    x, nn, sp, sn = node_targets(surf)
    xo, no = offsurface_targets(surf, rng, count_per_patch=per_patch, rel_dist=(1e-4, 0.5))
    xyz = np.concatenate([x, xo], axis=1)
    nrm = np.concatenate([nn, no], axis=1)
    sp = np.concatenate([sp, np.full(xo.shape[1], -1, np.int32)])
    sn = np.concatenate([sn, np.full(xo.shape[1], -1, np.int32)])
    tg = make_targets(surf, xyz, nrm, sp, sn, eta=1.5)
    return surf, tg, None


def quadratic_patch(k=(0.35, -0.2, 0.25), scale=0.6, shift=(0.0, 0.0, 0.0)):
    """One curved patch r(u, v) = scale (u, v, k0 u^2 + k1 u v + k2 v^2) + shift; its edges are
    quadratic curves, so the edge interpolants reproduce them exactly."""
    def fn(u, v):
        return (scale * u + shift[0], scale * v + shift[1],
                scale * (k[0] * u * u + k[1] * u * v + k[2] * v * v) + shift[2])
    return PatchMap(fn)


def paraboloid_patches(cases, q, spacing=10.0):
    """Quadrilateral pieces of the paraboloid z = H/2 (x^2 + y^2) over [-h/2, h/2]^2 (maximum
    mean curvature H, at the origin), one patch per (H, h) in `cases`, moved apart along x
    so that no target is near two of them."""
    maps = [quadratic_patch(k=(H * h / 4.0, 0.0, H * h / 4.0), scale=h / 2.0,
                            shift=(spacing * i, 0.0, 0.0)) for i, (H, h) in enumerate(cases)]
    return discretize(maps, np.full(len(cases), q))


def paraboloid_workload(cases, q=8, seed=SEED_BASE + 50):
    """Paraboloid patches with their node targets and 8 off-surface targets per patch at
    1e-3 .. 0.3 patch diameters.  Near radius 2.5 corner diameters: the corners of the most
    curved piece sit high above its bottom, so one diameter from their mean would miss the
    patch's own nodes."""
    rng = np.random.default_rng(seed)
    surf = paraboloid_patches(cases, q)
    x, nn, sp, sn = node_targets(surf)
    xo, no = offsurface_targets(surf, rng, count_per_patch=8, rel_dist=(1e-3, 0.3))
    m = xo.shape[1]
    tg = make_targets(surf, np.concatenate([x, xo], axis=1), np.concatenate([nn, no], axis=1),
                      np.concatenate([sp, np.full(m, -1, np.int32)]),
                      np.concatenate([sn, np.full(m, -1, np.int32)]), eta=2.5)
    return surf, tg


def patch_point(surface, P, u, v):
    """Point, unit normal of patch P at parameters (u, v)."""
    r, ru, rv = surface["maps"][P].derivs(np.atleast_1d(u), np.atleast_1d(v))
    n = np.cross(ru, rv)
    n /= np.linalg.norm(n, axis=1)[:, None]
    return r[0], n[0]
