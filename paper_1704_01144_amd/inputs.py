"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks: graded tetrahedral meshes and blast initial states.

This module holds no arithmetic of the method itself (no fluxes, gradients,
levels or schedules); it only produces node coordinates, tetrahedra and
primitive initial states, as plain NumPy arrays.

Meshes: an nx*ny*nz hex grid whose coordinates are graded geometrically,
x_k = (r^k - 1)/(r^n - 1) with r = G^(1/(n-1)) so that the last cell edge is
G times the first ("grading ratio G end to end"), each hex split into the 6
Kuhn tetrahedra along its (0,0,0)-(1,1,1) diagonal (a conforming split).
Cell order is structured: tet t of hex (i, j, k) has id ((k*ny + j)*nx + i)*6 + t.
"""
import itertools

import numpy as np

GAMMA = 1.4


def graded_coords(n, grading=1.0, length=1.0):
    """n+1 node coordinates on [0, length], edge ratio last/first = grading."""
    k = np.arange(n + 1, dtype=np.float64)
    if n < 2 or grading == 1.0:
        return length * k / n
    r = grading ** (1.0 / (n - 1))
    return length * (r ** k - 1.0) / (r ** n - 1.0)


# the 6 Kuhn tets: for each permutation s of the axes, the path
# (0,0,0) -> e_s0 -> e_s0 + e_s1 -> (1,1,1)
_KUHN = []
for perm in itertools.permutations(range(3)):
    v = [0, 0, 0]
    path = [tuple(v)]
    for ax in perm:
        v[ax] = 1
        path.append(tuple(v))
    _KUHN.append(path)


def kuhn_tet_mesh(xs, ys, zs):
    """Tetrahedral mesh of the tensor grid xs x ys x zs; returns
    (nodes[n_nodes][3] float64, tets[n_tets][4] int64), positively oriented."""
    xs, ys, zs = (np.asarray(a, dtype=np.float64) for a in (xs, ys, zs))
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    # node id = (k*(ny+1) + j)*(nx+1) + i
    nodes = np.stack([X.transpose(2, 1, 0).ravel(), Y.transpose(2, 1, 0).ravel(),
                      Z.transpose(2, 1, 0).ravel()], axis=1)
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    i, j, k = (a.transpose(2, 1, 0).ravel() for a in (i, j, k))  # hex order k, j, i

    def nid(di, dj, dk):
        return ((k + dk) * (ny + 1) + (j + dj)) * (nx + 1) + (i + di)

    tets = np.empty((nx * ny * nz, 6, 4), dtype=np.int64)
    for t, path in enumerate(_KUHN):
        for m, (di, dj, dk) in enumerate(path):
            tets[:, t, m] = nid(di, dj, dk)
    tets = tets.reshape(-1, 4)
    # orient: swap the last two vertices where the signed volume is negative
    p = nodes[tets]
    det = np.einsum("ij,ij->i", p[:, 1] - p[:, 0], np.cross(p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]))
    neg = det < 0
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    return nodes, tets


def graded_box_mesh(nx, ny, nz, grading):
    """nx x ny x nz hexes on the unit cube, each axis graded toward 0 with
    last/first edge ratio `grading`."""
    return kuhn_tet_mesh(graded_coords(nx, grading), graded_coords(ny, grading),
                         graded_coords(nz, grading))


def graded_cube_mesh(n, grading):
    """n^3 hexes on the unit cube, graded toward the origin in x, y and z."""
    x = graded_coords(n, grading)
    return kuhn_tet_mesh(x, x, x)


def column_mesh(n, grading=1.0, length=1.0, width=None):
    """A column of n x 1 x 1 hexes along x (shock-tube tests); the square
    cross section has edge `width` (default length/n)."""
    x = graded_coords(n, grading, length)
    h = length / n if width is None else width
    return kuhn_tet_mesh(x, np.array([0.0, h]), np.array([0.0, h]))


def tet_centroids(nodes, tets):
    return nodes[tets].mean(axis=1)


def blast_centre(seed):
    """Blast centre jittered uniformly in [0.3, 0.7]^3 from a seeded generator."""
    return np.random.default_rng(seed).uniform(0.3, 0.7, 3)


def blast_state(nodes, tets, centre=(0.5, 0.5, 0.5), radius=0.2, p_in=10.0, p_out=1.0,
                rho=1.0):
    """Primitive state [n_tets][5] = (rho, u, v, w, p): rho everywhere, at rest,
    p_in where the tet centroid lies strictly within `radius` of `centre`."""
    c = tet_centroids(nodes, tets)
    r = np.linalg.norm(c - np.asarray(centre, dtype=np.float64), axis=1)
    prim = np.zeros((len(tets), 5))
    prim[:, 0] = rho
    prim[:, 4] = np.where(r < radius, p_in, p_out)
    return prim


def random_state(n, seed, rho=(0.5, 2.0), vel=0.5, p=(0.5, 2.0)):
    """Smooth-free random primitive state (tests): uniform draws per cell."""
    g = np.random.default_rng(seed)
    prim = np.empty((n, 5))
    prim[:, 0] = g.uniform(*rho, n)
    prim[:, 1:4] = g.uniform(-vel, vel, (n, 3))
    prim[:, 4] = g.uniform(*p, n)
    return prim


def pulse_state(nodes, tets, centre=(0.5, 0.5, 0.5), width=0.2, amp=0.01,
                velocity=(0.1, 0.0, 0.0), rho=1.0, p=1.0, gamma=1.4):
    """Smooth state for convergence studies: a Gaussian bump
    g = exp(-|x - centre|^2 / width^2) of relative amplitude amp in density
    and gamma * amp in pressure (isentropic to first order) on a uniform
    flow of the given velocity."""
    c = tet_centroids(nodes, tets)
    g = np.exp(-((c - np.asarray(centre, dtype=np.float64)) ** 2).sum(1) / width ** 2)
    prim = np.zeros((len(tets), 5))
    prim[:, 0] = rho * (1.0 + amp * g)
    prim[:, 1:4] = np.asarray(velocity, dtype=np.float64)
    prim[:, 4] = p * (1.0 + gamma * amp * g)
    return prim


def motion_field(nodes, amp=0.05, seed=0, modes=3):
    """Smooth node velocities [n_nodes][3] for moving-mesh runs: per
    component a sum of `modes` plane sine waves amp * a * sin(2 pi k . x + c)
    with k, a, c drawn from default_rng(seed) (|k| up to 2, a in [-1, 1])."""
    rng = np.random.default_rng(seed)
    x = np.asarray(nodes, dtype=np.float64)
    v = np.zeros_like(x)
    for d in range(3):
        for _ in range(modes):
            k = rng.uniform(-2.0, 2.0, 3)
            a = rng.uniform(-1.0, 1.0)
            c = rng.uniform(0.0, 2.0 * np.pi)
            v[:, d] += amp * a * np.sin(2.0 * np.pi * (x @ k) + c)
    return v


def sod_state(nodes, tets, x0=0.5, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1)):
    """Shock-tube state along x: (rho, u, p) left of x0, right of it
    (Sod's 1978 data by default), zero transverse velocity."""
    c = tet_centroids(nodes, tets)
    prim = np.zeros((len(tets), 5))
    lft = c[:, 0] < x0
    prim[:, 0] = np.where(lft, left[0], right[0])
    prim[:, 1] = np.where(lft, left[1], right[1])
    prim[:, 4] = np.where(lft, left[2], right[2])
    return prim


def mlp_init(seed, n_in=6, n_h=32):
    """He-uniform initial parameters of the 6-32-32-1 guess network (biases
    0) as float32, in the library's order W1, b1, W2, b2, w3, b3."""
    rng = np.random.default_rng(seed)
    lim1, lim2 = np.sqrt(6.0 / n_in), np.sqrt(6.0 / n_h)
    parts = [rng.uniform(-lim1, lim1, (n_h, n_in)).ravel(), np.zeros(n_h),
             rng.uniform(-lim2, lim2, (n_h, n_h)).ravel(), np.zeros(n_h),
             rng.uniform(-lim2, lim2, n_h), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


# --- the configurations of the benchmark and the parity tests ------------

def config_small():
    """12^3 hexes, grading 4, 6 tets each (10,368 cells): first order, 3
    levels, 8 dt_min units, blast centred at (0.5, 0.5, 0.5)."""
    nodes, tets = graded_cube_mesh(12, 4.0)
    return dict(nodes=nodes, tets=tets, prim=blast_state(nodes, tets),
                order=1, max_levels=3, units=8)


def config_scale(n=64, seed=0):
    """n^3 hexes, grading 16, 6 tets each (n = 64: 1,572,864 cells): second
    order, 5 levels, 32 dt_min units, blast centre drawn from `seed`."""
    nodes, tets = graded_cube_mesh(n, 16.0)
    return dict(nodes=nodes, tets=tets,
                prim=blast_state(nodes, tets, centre=blast_centre(seed)),
                order=2, max_levels=5, units=32)


def batch_case(m, seed0=1000, size_range=(5000, 400000), grading_range=(2.0, 32.0),
               levels=(1, 6)):
    """Mesh m of the batched workload, from default_rng(seed0 + m): a target
    size log-uniform in size_range, grading log-uniform in grading_range, a
    level cap uniform over levels, a blast centre uniform in [0.3, 0.7]^3;
    n = round(cbrt(size / 6)) hexes along x and y and
    max(1, round(size / (6 n^2))) along z.  Returns a dict with nodes, tets,
    prim, max_levels, grading and the seed."""
    g = np.random.default_rng(seed0 + m)
    size = float(np.exp(g.uniform(np.log(size_range[0]), np.log(size_range[1]))))
    grading = float(np.exp(g.uniform(np.log(grading_range[0]), np.log(grading_range[1]))))
    L = int(g.integers(levels[0], levels[1] + 1))
    centre = g.uniform(0.3, 0.7, 3)
    n = max(1, int(round((size / 6.0) ** (1.0 / 3.0))))
    nz = max(1, int(round(size / (6.0 * n * n))))
    nodes, tets = graded_box_mesh(n, n, nz, grading)
    return dict(nodes=nodes, tets=tets, prim=blast_state(nodes, tets, centre=centre),
                max_levels=L, grading=grading, seed=seed0 + m, dims=(n, n, nz))


def config_batch(count=128, seed0=1000, **kw):
    """The batched workload: `count` meshes from batch_case(m) (128 meshes:
    about 11 million cells), FP32 flux, 16 dt_min units."""
    return [batch_case(m, seed0, **kw) for m in range(count)]
