"""Procedural triangle meshes for the synthetic CRSH workloads.

Seeded input generation only: nothing here computes any step of the
secondary-ray path.  Every mesh is returned as (vertices float64 [V,3],
faces int64 [F,3]); placement and rounding to float32 happen in
``workloads.scenes``.
"""
import numpy as np


def icosphere(subdiv):
    """Unit icosphere: 20 * 4**subdiv faces (subdivision 2 -> 320, 3 -> 1280)."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = list(f)
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts), np.array(faces, dtype=np.int64)


def torus(nu, nv, R=1.0, r=0.35):
    """Torus in the xz plane with nu x nv quads -> 2*nu*nv triangles."""
    i = np.arange(nu)
    j = np.arange(nv)
    a = 2.0 * np.pi * i / nu
    b = 2.0 * np.pi * j / nv
    A, Bm = np.meshgrid(a, b, indexing="ij")
    x = (R + r * np.cos(Bm)) * np.cos(A)
    z = (R + r * np.cos(Bm)) * np.sin(A)
    y = r * np.sin(Bm)
    verts = np.stack([x, y, z], -1).reshape(-1, 3)
    I, J = np.meshgrid(i, j, indexing="ij")
    p00 = I * nv + J
    p10 = ((I + 1) % nu) * nv + J
    p01 = I * nv + (J + 1) % nv
    p11 = ((I + 1) % nu) * nv + (J + 1) % nv
    f1 = np.stack([p00, p10, p11], -1).reshape(-1, 3)
    f2 = np.stack([p00, p11, p01], -1).reshape(-1, 3)
    faces = np.empty((2 * nu * nv, 3), dtype=np.int64)
    faces[0::2] = f1
    faces[1::2] = f2
    return verts, faces


def value_noise3(rng, freq=2.0, lattice=8):
    """Seeded trilinear value noise in [-1, 1] over R^3 (periodic lattice)."""
    table = rng.uniform(-1.0, 1.0, size=(lattice, lattice, lattice))

    def f(p):
        q = np.asarray(p, dtype=np.float64) * freq
        q0 = np.floor(q)
        w = q - q0
        w = w * w * (3.0 - 2.0 * w)
        i0 = q0.astype(np.int64) % lattice
        i1 = (i0 + 1) % lattice
        out = np.zeros(q.shape[:-1])
        for dx in (0, 1):
            wx = w[..., 0] if dx else 1.0 - w[..., 0]
            ix = i1[..., 0] if dx else i0[..., 0]
            for dy in (0, 1):
                wy = w[..., 1] if dy else 1.0 - w[..., 1]
                iy = i1[..., 1] if dy else i0[..., 1]
                for dz in (0, 1):
                    wz = w[..., 2] if dz else 1.0 - w[..., 2]
                    iz = i1[..., 2] if dz else i0[..., 2]
                    out = out + wx * wy * wz * table[ix, iy, iz]
        return out

    return f


def displaced_grid(n, rng, amp=0.15):
    """n x n quads over [-1,1]^2 in xz, heights from seeded value noise."""
    noise = value_noise3(rng, freq=1.5)
    g = np.linspace(-1.0, 1.0, n + 1)
    X, Z = np.meshgrid(g, g, indexing="ij")
    P = np.stack([X, np.zeros_like(X), Z], -1)
    Y = amp * noise(P + 0.37)
    verts = np.stack([X, Y, Z], -1).reshape(-1, 3)
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    p00 = I * (n + 1) + J
    p10 = (I + 1) * (n + 1) + J
    p01 = I * (n + 1) + J + 1
    p11 = (I + 1) * (n + 1) + J + 1
    faces = np.empty((2 * n * n, 3), dtype=np.int64)
    faces[0::2] = np.stack([p00, p10, p11], -1).reshape(-1, 3)
    faces[1::2] = np.stack([p00, p11, p01], -1).reshape(-1, 3)
    return verts, faces


def quad_grid(origin, eu, ev, nu, nv):
    """Planar grid origin + a*eu + b*ev, a,b in [0,1], nu x nv quads."""
    origin = np.asarray(origin, dtype=np.float64)
    eu = np.asarray(eu, dtype=np.float64)
    ev = np.asarray(ev, dtype=np.float64)
    a = np.linspace(0.0, 1.0, nu + 1)
    b = np.linspace(0.0, 1.0, nv + 1)
    A, Bm = np.meshgrid(a, b, indexing="ij")
    verts = origin + A[..., None] * eu + Bm[..., None] * ev
    verts = verts.reshape(-1, 3)
    I, J = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    p00 = I * (nv + 1) + J
    p10 = (I + 1) * (nv + 1) + J
    p01 = I * (nv + 1) + J + 1
    p11 = (I + 1) * (nv + 1) + J + 1
    faces = np.empty((2 * nu * nv, 3), dtype=np.int64)
    faces[0::2] = np.stack([p00, p10, p11], -1).reshape(-1, 3)
    faces[1::2] = np.stack([p00, p11, p01], -1).reshape(-1, 3)
    return verts, faces


def room_walls(lo, hi, sub):
    """Six inward walls of the box [lo, hi], each an sub x sub quad grid."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    ex = np.array([hi[0] - lo[0], 0, 0])
    ey = np.array([0, hi[1] - lo[1], 0])
    ez = np.array([0, 0, hi[2] - lo[2]])
    walls = [
        (lo, ex, ez),                      # floor
        (lo + ey, ez, ex),                 # ceiling
        (lo, ey, ex),                      # back (z = lo)
        (lo + ez, ex, ey),                 # front (z = hi)
        (lo, ez, ey),                      # left (x = lo)
        (lo + ex, ey, ez),                 # right (x = hi)
    ]
    return [quad_grid(o, u, v, sub, sub) for o, u, v in walls]


def random_rotation(rng):
    """Haar-uniform rotation matrix from a random unit quaternion (Shoemake)."""
    u1, u2, u3 = rng.uniform(0.0, 1.0, size=3)
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    x, y = a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2)
    z, w = b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])
