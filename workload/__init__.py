"""Seeded synthetic workloads shared by the solver and by its checker.

Everything here is input data: vertex coordinates and element-to-vertex
topology of a tetrahedral mesh of the unit cube, per-element wavespeeds,
random coefficient vectors, analytic initial fields, and the named workload
presets.  Nothing here evaluates a basis, a geometric factor, a flux or a
time step; each consumer derives those itself.

Meshes: [0,1]^3 is cut into n^3 cubes of edge h = 1/n and every cube into the
six Kuhn tetrahedra (one per ordering of the axes), which gives a conforming
mesh.  Interior vertices may be jittered uniformly by +-jitter*h per
coordinate; boundary vertices stay on the cube faces so the domain is exact.
"""
import itertools

import numpy as np

# Fixed seeds of every random draw in the workloads.
SEED_JITTER = 1001
SEED_WAVESPEED = 1002
SEED_SOURCES = 1003
SEED_FD_ELEMENTS = 1004
SEED_COEFFS = 1005


def kuhn_cube_mesh(n, jitter=0.0, seed=SEED_JITTER, drop_last=0):
    """Return (VX, EToV) for the unit cube split into 6*n^3 Kuhn tetrahedra.

    VX: float64 (Nv, 3) vertex coordinates.  EToV: int32 (K, 4) vertex ids;
    every tetrahedron is listed with positive orientation (the edge vectors
    v1-v0, v2-v0, v3-v0 form a right-handed triple).  Elements are ordered
    cube by cube (x fastest, then y, then z), six per cube.
    drop_last removes the last elements (their faces become boundary faces),
    which gives element counts that are not a multiple of 6.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    h = 1.0 / n
    g = np.arange(n + 1) * h
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    VX = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.float64)

    def vid(i, j, k):
        return i + (n + 1) * (j + (n + 1) * k)

    perms = list(itertools.permutations(range(3)))
    tets = []
    for k in range(n):
        for j in range(n):
            for i in range(n):
                base = np.array([i, j, k])
                for p in perms:
                    path = [base.copy()]
                    cur = base.copy()
                    for axis in p:
                        cur = cur.copy()
                        cur[axis] += 1
                        path.append(cur)
                    ids = [vid(*c) for c in path]
                    # odd axis orderings give a left-handed path: swap the last two
                    inversions = sum(1 for a in range(3) for b in range(a + 1, 3) if p[a] > p[b])
                    if inversions % 2 == 1:
                        ids[2], ids[3] = ids[3], ids[2]
                    tets.append(ids)
    EToV = np.asarray(tets, dtype=np.int32)
    if drop_last:
        if drop_last >= EToV.shape[0]:
            raise ValueError("drop_last removes every element")
        EToV = EToV[: EToV.shape[0] - drop_last]

    if jitter:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-jitter * h, jitter * h, size=VX.shape)
        on_boundary = np.any((np.abs(VX) < 1e-12) | (np.abs(VX - 1.0) < 1e-12), axis=1)
        d[on_boundary] = 0.0
        VX = VX + d
    return VX, EToV


def wavespeed(K, lo=1.0, hi=1.0, seed=SEED_WAVESPEED):
    """Per-element wavespeed c (float64, K): constant if lo == hi, else U[lo, hi]."""
    if lo == hi:
        return np.full(K, float(lo))
    return np.random.default_rng(seed).uniform(lo, hi, size=K)


def random_coeffs(K, Np, seed=SEED_COEFFS, nfields=4):
    """Standard-normal coefficient array of shape (nfields, K, Np), float64."""
    return np.random.default_rng(seed).standard_normal((nfields, K, Np))


def standing_mode_p0(x, y, z):
    """Initial pressure cos(pi x) cos(pi y) cos(pi z) (velocity starts at zero)."""
    return np.cos(np.pi * x) * np.cos(np.pi * y) * np.cos(np.pi * z)


def gaussian_pulse_p0(x, y, z, width=100.0, centre=(0.5, 0.5, 0.5)):
    """Initial pressure exp(-width |x - centre|^2) (velocity starts at zero)."""
    return np.exp(-width * ((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2))


def zero_p0(x, y, z):
    return np.zeros_like(x)


INITIAL_FIELDS = {
    "standing_mode": standing_mode_p0,
    "gaussian_pulse": gaussian_pulse_p0,
    "zero": zero_p0,
}


def nodes_per_element(N):
    return (N + 1) * (N + 2) * (N + 3) // 6


# Named workloads.  dt follows dt = 0.5 h / (c_max (N+1)^2).
PRESETS = {
    # 384 tets, N=3, c=1, standing mode, rigid walls, 10 steps
    "c1": dict(n=4, jitter=0.0, N=3, c=(1.0, 1.0), ic="standing_mode", steps=10),
    # 24,576 jittered tets, N=5, c=1, standing mode, 1000 steps
    "c2": dict(n=16, jitter=0.1, N=5, c=(1.0, 1.0), ic="standing_mode", steps=1000),
    # 196,608 tets, N in {1,3,5,7,9}, c ~ U[1,3], Gaussian pulse, 200 steps
    "c3": dict(n=32, jitter=0.0, N=5, c=(1.0, 3.0), ic="gaussian_pulse", steps=200),
    # 24,576 tets, N=4, c ~ U[1,3], 64 shots (Ricker point sources f0 = 8,
    # delay 1/f0, seeded positions in [0.1, 0.9]^3), 8 x 8 receivers on
    # z = 0.9, zero initial state, 500 steps
    "c4": dict(n=16, jitter=0.0, N=4, c=(1.0, 3.0), ic="zero", steps=500, shots=64, f0=8.0, ts=0.125),
    # 24,576 tets, N=5, misfit gradient: 8 shots with Ricker sources on the
    # plane z = 0.9, 8 x 8 receivers on the same plane, observations from the
    # blob model m_true, gradient at m = 1, 500 steps, checkpoints every 50
    "c5": dict(n=16, jitter=0.0, N=5, c=(1.0, 1.0), ic="zero", steps=500, shots=8, f0=8.0, ts=0.125,
               ckpt_every=50),
}


def preset(name, **overrides):
    """Return a dict describing a named workload, with dt filled in."""
    cfg = dict(PRESETS[name])
    cfg.update(overrides)
    h = 1.0 / cfg["n"]
    cmax = max(cfg["c"])
    cfg["h"] = h
    cfg["dt"] = 0.5 * h / (cmax * (cfg["N"] + 1) ** 2)
    cfg["K"] = 6 * cfg["n"] ** 3
    cfg["Np"] = nodes_per_element(cfg["N"])
    return cfg


def build_preset(name, **overrides):
    """Return (cfg, VX, EToV, c) for a named workload."""
    cfg = preset(name, **overrides)
    VX, EToV = kuhn_cube_mesh(cfg["n"], cfg["jitter"])
    c = wavespeed(EToV.shape[0], *cfg["c"])
    return cfg, VX, EToV, c


def source_positions(S, seed=SEED_SOURCES, lo=0.1, hi=0.9):
    """(S, 3) point-source positions, uniform in [lo, hi]^3."""
    return np.random.default_rng(seed).uniform(lo, hi, (S, 3))


def receiver_grid(m=8, z=0.9, lo=0.1, hi=0.9):
    """(m*m, 3) receivers on an m x m grid of the plane z, x and y in [lo, hi]."""
    t = lo + (hi - lo) * np.arange(m) / (m - 1)
    X, Y = np.meshgrid(t, t, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), np.full(m * m, z)], axis=1)


def plane_sources(S, z=0.9, seed=SEED_SOURCES, lo=0.1, hi=0.9):
    """(S, 3) source positions uniform in [lo, hi]^2 on the plane z."""
    xy = np.random.default_rng(seed).uniform(lo, hi, (S, 2))
    return np.concatenate([xy, np.full((S, 1), z)], axis=1)


def blob_model(VX, EToV, centre=(0.5, 0.5, 0.75), amp=0.5, width=100.0):
    """m = c^2 per element: 1 + amp exp(-width |x_k - centre|^2) at the element centroids."""
    cen = np.asarray(VX)[np.asarray(EToV)].mean(axis=1)
    r2 = np.sum((cen - np.asarray(centre)) ** 2, axis=1)
    return 1.0 + amp * np.exp(-width * r2)


def element_count(n, drop_last=0):
    return 6 * n ** 3 - drop_last


__all__ = [
    "kuhn_cube_mesh", "wavespeed", "random_coeffs", "standing_mode_p0",
    "gaussian_pulse_p0", "INITIAL_FIELDS", "PRESETS", "preset", "build_preset",
    "nodes_per_element", "element_count", "source_positions", "receiver_grid", "plane_sources", "blob_model",
]
