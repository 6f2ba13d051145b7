"""crsh_hash_static, the allocation-free form of crsh_hash (its scratch is a
static device array): the same rays, keys and ids as crsh_hash on two calls
in a row, the second on a smaller frame than the first, and host-side
rejection of frames beyond the array's size."""
import ctypes

import numpy as np
import pytest

from conftest import workload
from paper_2312_06538_amd import crsh as X

SIZES = [("refl_1024", dict(W=320, H=240)), ("shadow_128", dict(W=64, H=48))]


def test_static_hash_rejects_frames_beyond_its_scratch():
    L = X.lib()
    side = 1 << 13                                  # 2^26 pixels > 2^25
    g = X.Gbuf(*([1] * 7), side, side)
    rg = X.Raygen()
    r = X.Rays(*([1] * 8), 100)
    assert L.crsh_hash_static(ctypes.byref(g), ctypes.byref(rg), ctypes.byref(r), 1, 1, 1, None) == X.ERR_INVALID
    assert "exceed" in X.last_error()
    assert L.crsh_hash_static(None, ctypes.byref(rg), ctypes.byref(r), 1, 1, 1, None) == X.ERR_INVALID


@pytest.mark.gpu
def test_static_hash_matches_crsh_hash_on_consecutive_calls():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_06538_amd import pipeline as P
    import gpu_util as gu

    def buffers(fr):
        cap = fr.max_rays
        rays = {k: torch.full((cap,), -7.0, dtype=torch.float32, device="cuda") for k in P.RAY_KEYS}
        rays["pix"] = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
        keys = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
        ids = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
        c = X.Rays(*[rays[k].data_ptr() for k in P.RAY_KEYS], rays["pix"].data_ptr(), cap)
        return rays, keys, ids, c

    def host(rays, keys, ids, meta):
        m, st = gu.read_meta(meta)
        assert st == X.OK, X.last_error()
        n = int(m.n_rays)
        out = {k: rays[k][:n].cpu().numpy().view(np.uint32) for k in P.RAY_KEYS}
        out["pix"] = P.u32(rays["pix"][:n])
        out["keys"] = P.u32(keys[:n])
        out["ids"] = P.u32(ids[:n])
        return n, out

    frames = []
    for name, kw in SIZES:
        wl = workload(name, **kw)
        frames.append(P.DeviceFrame(wl))
    assert frames[1].W * frames[1].H < frames[0].W * frames[0].H
    # two static calls in a row (the second on the smaller frame, so the
    # array still holds the first call's larger count table)
    static = []
    for fr in frames:
        rays, keys, ids, c = buffers(fr)
        meta = gu.new_meta()
        print(f"[no-alloc] crsh_hash_static {fr.W}x{fr.H}", flush=True)
        X.crsh_hash_static(fr.gbuf, fr.raygen, c, keys.data_ptr(), ids.data_ptr(), meta.data_ptr(), gu.s())
        static.append(host(rays, keys, ids, meta))
    for fr, (n, got) in zip(frames, static):
        rays, keys, ids, c = buffers(fr)
        meta = gu.new_meta()
        wsb = X.crsh_workspace_size(fr.max_rays, 1, 1, 1, 1)
        ws = gu.ws_tensor(wsb)
        X.crsh_hash(fr.gbuf, fr.raygen, c, keys.data_ptr(), ids.data_ptr(), meta.data_ptr(), ws.data_ptr(), wsb,
                    gu.s())
        n_ref, ref = host(rays, keys, ids, meta)
        assert n == n_ref and n > 0, (fr.W, fr.H, n, n_ref)
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (fr.W, fr.H, k)
        print(f"[no-alloc] {fr.W}x{fr.H}: {n} rays equal", flush=True)
