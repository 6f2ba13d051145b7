"""Primary visibility for the synthetic workloads (the primary-hit buffer).

The paper obtains primary hits by rasterization (Sec. 3.2: position, normal
and material per pixel in 32-bit float render targets).  Here they come from
casting one ray through every pixel centre in float64 on the host, so both
the oracle and the GPU path read the same buffer.  The candidate triangles of
a pixel are found from each triangle's screen bounding box (after clipping at
the near plane); each candidate is then tested exactly with a ray-plane
intersection and three edge-side tests.  Nearest hit wins, ties go to the
lower triangle id.

Input generation only: no step of the secondary-ray path lives here.
"""
import numpy as np

NEAR = 1e-4


def _cross(a, b):
    """Row-wise cross product of two [N,3] float64 arrays (the same products
    and differences as np.cross, without its copies)."""
    a0, a1, a2 = a[:, 0], a[:, 1], a[:, 2]
    b0, b1, b2 = b[:, 0], b[:, 1], b[:, 2]
    c = np.empty(a.shape, dtype=np.float64)
    c[:, 0] = a1 * b2 - a2 * b1
    c[:, 1] = a2 * b0 - a0 * b2
    c[:, 2] = a0 * b1 - a1 * b0
    return c


def camera_basis(eye, look, up=(0.0, 1.0, 0.0)):
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(look, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, dtype=np.float64))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    return f, r, u


def pixel_dirs(W, H, eye, look, vfov_deg):
    """Unit float64 directions through the pixel centres, row-major, row 0 on top."""
    f, r, u = camera_basis(eye, look)
    th = np.tan(np.radians(vfov_deg) / 2.0)
    aspect = W / H
    xs = ((np.arange(W) + 0.5) / W * 2.0 - 1.0) * th * aspect
    ys = (1.0 - (np.arange(H) + 0.5) / H * 2.0) * th
    d = f[None, None, :] + xs[None, :, None] * r[None, None, :] + ys[:, None, None] * u[None, None, :]
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return d.reshape(-1, 3)


def _screen_bboxes(tris, W, H, eye, look, vfov_deg):
    """Pixel bounding box [x0,x1]x[y0,y1] of each triangle's visible part (-1 if none)."""
    f, r, u = camera_basis(eye, look)
    th = np.tan(np.radians(vfov_deg) / 2.0)
    aspect = W / H
    rel = tris - np.asarray(eye, dtype=np.float64)[None, None, :]
    xv = rel @ r
    yv = rel @ u
    zv = rel @ f
    M = tris.shape[0]
    box = np.full((M, 4), -1, dtype=np.int64)

    def to_px(x, y, z):
        sx = ((x / z) / (th * aspect) + 1.0) * 0.5 * W - 0.5
        sy = (1.0 - (y / z) / th) * 0.5 * H - 0.5
        return sx, sy

    front = zv > NEAR
    allf = front.all(axis=1)
    if allf.any():
        sx, sy = to_px(xv[allf], yv[allf], zv[allf])
        box[allf, 0] = np.floor(sx.min(1)).astype(np.int64) - 1
        box[allf, 1] = np.ceil(sx.max(1)).astype(np.int64) + 1
        box[allf, 2] = np.floor(sy.min(1)).astype(np.int64) - 1
        box[allf, 3] = np.ceil(sy.max(1)).astype(np.int64) + 1
    # triangles crossing the near plane: clip, then take the box of the clipped polygon
    for t in np.nonzero(front.any(axis=1) & ~allf)[0]:
        pts = []
        for a in range(3):
            b = (a + 1) % 3
            pa = (xv[t, a], yv[t, a], zv[t, a])
            pb = (xv[t, b], yv[t, b], zv[t, b])
            if pa[2] > NEAR:
                pts.append(pa)
            if (pa[2] > NEAR) != (pb[2] > NEAR):
                s = (NEAR - pa[2]) / (pb[2] - pa[2])
                pts.append((pa[0] + s * (pb[0] - pa[0]), pa[1] + s * (pb[1] - pa[1]), NEAR))
        P = np.array(pts)
        sx, sy = to_px(P[:, 0], P[:, 1], np.maximum(P[:, 2], NEAR))
        box[t] = [np.floor(sx.min()) - 1, np.ceil(sx.max()) + 1,
                  np.floor(sy.min()) - 1, np.ceil(sy.max()) + 1]
    vis = front.any(axis=1)
    vis &= (box[:, 1] >= 0) & (box[:, 0] <= W - 1) & (box[:, 3] >= 0) & (box[:, 2] <= H - 1)
    box[:, 0] = np.clip(box[:, 0], 0, W - 1)
    box[:, 1] = np.clip(box[:, 1], 0, W - 1)
    box[:, 2] = np.clip(box[:, 2], 0, H - 1)
    box[:, 3] = np.clip(box[:, 3], 0, H - 1)
    return box, vis


def cast_primary(tris32, tri_mat, W, H, eye, look, vfov_deg, chunk=4_000_000):
    """Nearest hit through each pixel centre.

    Returns dict with float32 px,py,pz (hit point), nx,ny,nz (unit geometric
    normal facing the camera), int32 mat (material, -1 = no hit) and int32 tri
    (hit triangle, -1 = no hit), all row-major of length W*H.
    """
    tris = tris32.astype(np.float64)
    eye64 = np.asarray(eye, dtype=np.float64)
    dirs = pixel_dirs(W, H, eye, look, vfov_deg)
    box, vis = _screen_bboxes(tris, W, H, eye, look, vfov_deg)
    ids = np.nonzero(vis)[0]
    area = (box[ids, 1] - box[ids, 0] + 1) * (box[ids, 3] - box[ids, 2] + 1)
    best_t = np.full(W * H, np.inf)
    best_tri = np.full(W * H, -1, dtype=np.int64)
    e1 = tris[:, 1] - tris[:, 0]
    e2 = tris[:, 2] - tris[:, 0]
    nrm = _cross(e1, e2)
    start = 0
    csum = np.cumsum(area)
    while start < len(ids):
        base = csum[start - 1] if start > 0 else 0
        stop = int(np.searchsorted(csum, base + chunk, side="right"))
        stop = max(stop, start + 1)
        tid = ids[start:stop]
        a = area[start:stop]
        tt = np.repeat(tid, a)
        local = np.arange(a.sum()) - np.repeat(np.cumsum(a) - a, a)
        bw = np.repeat(box[tid, 1] - box[tid, 0] + 1, a)
        px = np.repeat(box[tid, 0], a) + local % bw
        py = np.repeat(box[tid, 2], a) + local // bw
        pix = py * W + px
        d = dirs[pix]
        n = nrm[tt]
        den = np.einsum("ij,ij->i", d, n)
        v0 = tris[tt, 0]
        num = np.einsum("ij,ij->i", v0 - eye64, n)
        with np.errstate(divide="ignore", invalid="ignore"):
            t = num / den
        ok = (np.abs(den) > 0) & (t > 1e-9)
        h = eye64 + t[:, None] * d
        for k in range(3):
            va = tris[tt, k]
            vb = tris[tt, (k + 1) % 3]
            side = np.einsum("ij,ij->i", _cross(vb - va, h - va), n)
            ok &= side >= 0
        pix, t, tt = pix[ok], t[ok], tt[ok]
        order = np.lexsort((tt, t, pix))
        pix, t, tt = pix[order], t[order], tt[order]
        first = np.ones(len(pix), dtype=bool)
        first[1:] = pix[1:] != pix[:-1]
        pix, t, tt = pix[first], t[first], tt[first]
        better = (t < best_t[pix]) | ((t == best_t[pix]) & (tt < best_tri[pix]))
        best_t[pix[better]] = t[better]
        best_tri[pix[better]] = tt[better]
        start = stop
    hit = best_tri >= 0
    P = np.zeros((W * H, 3))
    N = np.zeros((W * H, 3))
    P[hit] = eye64 + best_t[hit, None] * dirs[hit]
    n = nrm[best_tri[hit]]
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    flip = np.einsum("ij,ij->i", n, dirs[hit]) > 0
    n[flip] = -n[flip]
    N[hit] = n
    mat = np.full(W * H, -1, dtype=np.int32)
    mat[hit] = tri_mat[best_tri[hit]]
    P32 = P.astype(np.float32)
    N32 = N.astype(np.float32)
    return {
        "px": np.ascontiguousarray(P32[:, 0]), "py": np.ascontiguousarray(P32[:, 1]),
        "pz": np.ascontiguousarray(P32[:, 2]),
        "nx": np.ascontiguousarray(N32[:, 0]), "ny": np.ascontiguousarray(N32[:, 1]),
        "nz": np.ascontiguousarray(N32[:, 2]),
        "mat": mat, "tri": best_tri.astype(np.int32),
    }
