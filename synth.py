"""Seeded synthetic inputs for the PIE/MLFMA workloads.

This module holds input generation only: sphere meshes, plane-wave
parameters, random coefficient vectors and the named workload shapes.  It
contains none of the method's arithmetic (no basis functions, no Green's
function, no quadrature, no tree).  Both the CPU oracle and the HIP path take
their inputs from here and from nowhere else.

Workloads stand in for the paper's sphere experiments (Section 4: a 0.6 m PEC
sphere illuminated by a z-travelling, x-polarised plane wave); the paper's own
meshes are not available, so icospheres of the same diameter are used.
"""
from __future__ import annotations

import dataclasses

import numpy as np

# Physical constants (SI).  Only the speed of light is needed here, to turn a
# diameter-to-wavelength ratio into a frequency.
C0 = 299792458.0
DIAMETER = 0.6  # metres, the sphere of Section 4


# ----------------------------------------------------------------------------
# SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
# generators", OOPSLA 2014): a counter-based stream; draw n of seed s is
# mix(s + (n + 1) * gamma).
# ----------------------------------------------------------------------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int) -> np.ndarray:
    """First ``n`` outputs of SplitMix64 started at ``seed`` (uint64 array)."""
    with np.errstate(over="ignore"):
        ctr = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed) + ctr * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix_uniform(seed: int, n: int) -> np.ndarray:
    """Uniform doubles in [0, 1): the top 53 bits of each SplitMix64 draw."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# ----------------------------------------------------------------------------
# Icosphere
# ----------------------------------------------------------------------------
def _icosahedron():
    g = (1.0 + 5.0 ** 0.5) / 2.0
    pts = []
    for a in (-1.0, 1.0):
        for b in (-g, g):
            pts += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    V = np.array(pts, dtype=np.float64)
    V /= np.linalg.norm(V, axis=1)[:, None]
    # faces = triples of mutually adjacent vertices (shortest chord)
    D = np.linalg.norm(V[:, None, :] - V[None, :, :], axis=2)
    e = np.min(D[D > 0])
    adj = np.abs(D - e) < 1e-9
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            if not adj[i, j]:
                continue
            for k in range(j + 1, 12):
                if adj[i, k] and adj[j, k]:
                    a, b, c = V[i], V[j], V[k]
                    if np.dot(np.cross(b - a, c - a), a + b + c) < 0.0:
                        faces.append((i, k, j))
                    else:
                        faces.append((i, j, k))
    F = np.array(faces, dtype=np.int64)
    assert F.shape == (20, 3)
    return V, F


def _subdivide(V, F):
    """Split every face into four; new midpoint vertices are appended in the
    order they are first created while walking faces and their edges
    (v0v1, v1v2, v2v0)."""
    nv = V.shape[0]
    ea = np.stack([F[:, 0], F[:, 1], F[:, 2]], axis=1).reshape(-1)
    eb = np.stack([F[:, 1], F[:, 2], F[:, 0]], axis=1).reshape(-1)
    lo = np.minimum(ea, eb)
    hi = np.maximum(ea, eb)
    key = lo * nv + hi
    uniq, first, inv = np.unique(key, return_index=True, return_inverse=True)
    order = np.argsort(first, kind="stable")
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    mid_id = nv + rank[inv]  # new vertex id per (face, edge)
    ulo, uhi = uniq // nv, uniq % nv
    M = V[ulo[order]] + V[uhi[order]]
    M = 0.5 * M
    M /= np.linalg.norm(M, axis=1)[:, None]
    mid = mid_id.reshape(-1, 3)  # m01, m12, m20
    v0, v1, v2 = F[:, 0], F[:, 1], F[:, 2]
    m01, m12, m20 = mid[:, 0], mid[:, 1], mid[:, 2]
    NF = np.stack([
        np.stack([v0, m01, m20], 1),
        np.stack([v1, m12, m01], 1),
        np.stack([v2, m20, m12], 1),
        np.stack([m01, m12, m20], 1),
    ], axis=1).reshape(-1, 3)
    return np.concatenate([V, M], axis=0), NF


def icosphere(subdiv: int, radius: float = DIAMETER / 2, jitter: float = 0.0,
              seed: int = 0):
    """Closed, outward-oriented (counter-clockwise seen from outside) sphere
    mesh with 20*4**subdiv triangles.

    ``jitter`` > 0 moves every vertex by jitter*h_v*(2u-1) per coordinate,
    where h_v is the shortest edge at that vertex on the unjittered mesh and u
    comes from SplitMix64(seed) drawn in vertex order, x then y then z.
    Returns (V float64 [nv,3], T int32 [nt,3]).
    """
    V, F = _icosahedron()
    for _ in range(subdiv):
        V, F = _subdivide(V, F)
    V = V * radius
    if jitter > 0.0:
        a = np.concatenate([F[:, 0], F[:, 1], F[:, 2]])
        b = np.concatenate([F[:, 1], F[:, 2], F[:, 0]])
        L = np.linalg.norm(V[a] - V[b], axis=1)
        h = np.full(V.shape[0], np.inf)
        np.minimum.at(h, a, L)
        np.minimum.at(h, b, L)
        u = splitmix_uniform(seed, 3 * V.shape[0]).reshape(-1, 3)
        V = V + jitter * h[:, None] * (2.0 * u - 1.0)
    return np.ascontiguousarray(V), np.ascontiguousarray(F.astype(np.int32))


# ----------------------------------------------------------------------------
# Open surfaces (flat plates in the plane z = 0, normal +z)
# ----------------------------------------------------------------------------
def patch(n: int, edge: float = DIAMETER, cross: bool = False):
    """Square plate [-edge/2, edge/2]^2 in z = 0 on an n x n grid of squares,
    counter-clockwise seen from +z.  Each square is split into two triangles
    along a diagonal whose direction alternates with (i + j) mod 2
    (2 n^2 triangles; n = 75 gives the 11 250 triangles of the paper's patch),
    or, with ``cross``, into four triangles around its centre (4 n^2
    triangles, symmetric under x -> -x, y -> -y and x <-> y).
    Returns (V float64 [nv,3], T int32 [nt,3])."""
    g = (np.arange(n + 1) / n - 0.5) * edge
    X, Y = np.meshgrid(g, g, indexing="ij")          # vertex (i, j) = i * (n + 1) + j
    V = [np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], 1)]
    vid = lambda i, j: i * (n + 1) + j
    T = []
    nc = (n + 1) ** 2
    for i in range(n):
        for j in range(n):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)  # ccw corners
            if cross:
                m = nc + i * n + j
                T += [(a, b, m), (b, c, m), (c, d, m), (d, a, m)]
            elif (i + j) % 2 == 0:
                T += [(a, b, c), (a, c, d)]
            else:
                T += [(a, b, d), (b, c, d)]
    if cross:
        cx = 0.5 * (g[:-1] + g[1:])
        CX, CY = np.meshgrid(cx, cx, indexing="ij")
        V.append(np.stack([CX.ravel(), CY.ravel(), np.zeros(CX.size)], 1))
    return np.ascontiguousarray(np.concatenate(V)), np.ascontiguousarray(np.array(T, dtype=np.int32))


def disk(rings: int, radius: float = DIAMETER / 2):
    """Circular plate of the given radius in z = 0, counter-clockwise seen
    from +z: a centre vertex and rings k = 1..rings of 6k vertices at radius
    radius * k / rings (angles 2 pi m / (6k)); neighbouring rings are joined
    by one strip of triangles, advancing on whichever ring's next vertex has
    the smaller angle.  6 rings^2 triangles.  Returns (V, T)."""
    V = [np.zeros((1, 3))]
    start = [0]
    for k in range(1, rings + 1):
        th = 2.0 * np.pi * np.arange(6 * k) / (6 * k)
        r = radius * k / rings
        start.append(sum(len(v) for v in V))
        V.append(np.stack([r * np.cos(th), r * np.sin(th), np.zeros(6 * k)], 1))
    T = []
    for m in range(6):                                  # centre fan
        T.append((0, 1 + m, 1 + (m + 1) % 6))
    for k in range(2, rings + 1):
        n0, n1, s0, s1 = 6 * (k - 1), 6 * k, start[k - 1], start[k]
        i0 = i1 = 0
        while i0 < n0 or i1 < n1:
            # angles of the next vertices (the ring closes at 1.0 = 2 pi)
            t0 = (i0 + 1) / n0 if i0 < n0 else 2.0
            t1 = (i1 + 1) / n1 if i1 < n1 else 2.0
            a0, a1 = s0 + i0 % n0, s1 + i1 % n1
            if t1 <= t0:
                T.append((a0, a1, s1 + (i1 + 1) % n1))
                i1 += 1
            else:
                T.append((a0, a1, s0 + (i0 + 1) % n0))
                i0 += 1
    return np.ascontiguousarray(np.concatenate(V)), np.ascontiguousarray(np.array(T, dtype=np.int32))


# ----------------------------------------------------------------------------
# Plane waves and coefficient vectors
# ----------------------------------------------------------------------------
def plane_waves(R: int, seed: int):
    """R seeded plane waves: directions uniform on the sphere
    (z = 2u1-1, phi = 2 pi u2) and polarisations cos(b) theta_hat +
    sin(b) phi_hat with b = 2 pi u3, from numpy's PCG64.
    Returns khat [R,3], pol [R,3] (unit, orthogonal), amp [R] complex (ones)."""
    rng = np.random.default_rng(seed)
    u = rng.random((R, 3))
    z = 2.0 * u[:, 0] - 1.0
    ph = 2.0 * np.pi * u[:, 1]
    st = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    khat = np.stack([st * np.cos(ph), st * np.sin(ph), z], 1)
    th_hat = np.stack([z * np.cos(ph), z * np.sin(ph), -st], 1)
    ph_hat = np.stack([-np.sin(ph), np.cos(ph), np.zeros(R)], 1)
    b = 2.0 * np.pi * u[:, 2]
    pol = np.cos(b)[:, None] * th_hat + np.sin(b)[:, None] * ph_hat
    return khat, pol, np.ones(R, dtype=np.complex128)


def axial_wave():
    """The paper's illumination: travelling along +z, polarised along x."""
    return (np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]),
            np.ones(1, dtype=np.complex128))


def complex_gaussian(n: int, R: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((n, R)) + 1j * rng.standard_normal((n, R)))


def sphere_directions(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    u = rng.random((n, 2))
    z = 2.0 * u[:, 0] - 1.0
    ph = 2.0 * np.pi * u[:, 1]
    st = np.sqrt(1.0 - z * z)
    return np.stack([st * np.cos(ph), st * np.sin(ph), z], 1)


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    subdiv: int                  # sphere: subdivisions; patch: squares per edge
    d_over_lambda: float         # sphere diameter or patch edge over the wavelength
    levels: int
    nrhs: int
    jitter: float = 0.0
    seed: int = 0
    rhs_seed: int | None = None  # None: the single axial wave
    shape: str = "sphere"        # "sphere" or "patch"

    @property
    def freq(self) -> float:
        return self.d_over_lambda * C0 / DIAMETER

    def mesh(self):
        if self.shape == "patch":
            return patch(self.subdiv, DIAMETER)
        return icosphere(self.subdiv, DIAMETER / 2, self.jitter, self.seed)

    def waves(self):
        if self.rhs_seed is None:
            return axial_wave()
        return plane_waves(self.nrhs, self.rhs_seed)


WORKLOADS = {
    # sphere D = 0.1 lambda, 1280 triangles, 3 levels (single-level FMM)
    "sphere_s3_0.1lam": Workload("sphere_s3_0.1lam", 3, 0.1, 3, 1),
    # sphere D = 1e-3 lambda, 20480 triangles, 5% vertex jitter, 5 levels
    "sphere_s5_1e-3lam_jit": Workload("sphere_s5_1e-3lam_jit", 5, 1e-3, 5, 1,
                                      jitter=0.05, seed=2),
    # sphere D = 1e-2 lambda, 81920 triangles, 64 plane waves, 6 levels
    "sphere_s6_1e-2lam_r64": Workload("sphere_s6_1e-2lam_r64", 6, 1e-2, 6, 64,
                                      rhs_seed=3),
    # sphere D = 1e-4 lambda, 20480 triangles, 16 plane waves, 5 levels
    "sphere_s5_1e-4lam_r16": Workload("sphere_s5_1e-4lam_r16", 5, 1e-4, 5, 16,
                                      rhs_seed=4),
    # the paper's patch: 0.6 m edge, 75 x 75 squares (11 250 triangles,
    # 16 725 RWG), axial wave, at 1 MHz (edge lambda/500) and 100 MHz
    # (lambda/5); 5 levels (finest boxes of about 4.7 mesh edges)
    "patch_75_1MHz": Workload("patch_75_1MHz", 75, 0.6 / (C0 / 1e6), 5, 1, shape="patch"),
    "patch_75_100MHz": Workload("patch_75_100MHz", 75, 0.6 / (C0 / 1e8), 5, 1, shape="patch"),
}


def uneven_batch():
    """Eight spheres, subdivisions {4,5,5,6,6,7,7,8}, D/lambda log-uniform in
    [1e-5, 1e-1] (PCG64 seed 5), 8 plane waves each (seed 50 + i)."""
    rng = np.random.default_rng(5)
    u = rng.random(8)
    out = []
    for i, s in enumerate((4, 5, 5, 6, 6, 7, 7, 8)):
        out.append(Workload(f"uneven_{i}_s{s}", s, 10.0 ** (-5.0 + 4.0 * u[i]),
                            s, 8, rhs_seed=50 + i))
    return out
