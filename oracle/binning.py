"""Tile binning implied by the definition: (view | tile | depth) keys.

The 3DGS rasterizer the paper keeps (Sec. 3.3) duplicates every visible
Gaussian once per screen tile its footprint touches and sorts the copies by a
key whose high part is the tile and whose low part is the depth; each tile
then composites its list front to back.  With views batched, tiles of view v
are numbered after those of views 0..v-1:

    tiles_x[v] = ceil(W_v / ts),  tiles_y[v] = ceil(H_v / ts)
    tile_base[v] = sum_{u < v} tiles_x[u] tiles_y[u]
    key = (tile_base[v] + ty * tiles_x[v] + tx) << 32 | zbits
    value = Gaussian index g

for every (tx, ty) in the FP32 tile rectangle of g, sorted ascending by
(key, value).  ``tile_csr`` is the exclusive prefix of the per-tile list
lengths (length T_total + 1).  Because the per-pixel candidate list is the
same (zbits, g) order filtered by the pixel box, each tile's list restricted
to a pixel is that pixel's candidate list; the tests check this.

Parity status: pinned by brute force (per-pixel candidate lists) on small
scenes.
"""
from __future__ import annotations

import numpy as np

from .spec32 import spec32


def tile_grid(cams, ts):
    tx = np.array([(c.width + ts - 1) // ts for c in cams], dtype=np.int64)
    ty = np.array([(c.height + ts - 1) // ts for c in cams], dtype=np.int64)
    base = np.concatenate([[0], np.cumsum(tx * ty)])
    return tx, ty, base


def tile_lists(scene, cams, ts):
    """Sorted keys (uint64), values (uint32 Gaussian index) and tile CSR."""
    tx_n, ty_n, base = tile_grid(cams, ts)
    keys_all, vals_all = [], []
    for v, cam in enumerate(cams):
        s = spec32(scene.mean, scene.log_scale, scene.quat, cam, ts)
        g = np.nonzero(s["visible"])[0]
        tx0, tx1, ty0, ty1 = (r[g].astype(np.int64) for r in s["rect"])
        wdt = tx1 - tx0 + 1
        cnt = wdt * (ty1 - ty0 + 1)
        rep = np.repeat(np.arange(len(g)), cnt)
        k = np.arange(int(cnt.sum())) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        tx = tx0[rep] + k % wdt[rep]
        ty = ty0[rep] + k // wdt[rep]
        tile = base[v] + ty * tx_n[v] + tx
        keys_all.append((tile.astype(np.uint64) << np.uint64(32)) | s["zbits"][g][rep].astype(np.uint64))
        vals_all.append(g[rep].astype(np.uint32))
    keys = np.concatenate(keys_all) if keys_all else np.zeros(0, np.uint64)
    vals = np.concatenate(vals_all) if vals_all else np.zeros(0, np.uint32)
    order = np.lexsort((vals, keys))
    keys, vals = keys[order], vals[order]
    tiles = (keys >> np.uint64(32)).astype(np.int64)
    csr = np.searchsorted(tiles, np.arange(int(base[-1]) + 1), side="left").astype(np.int64)
    return keys, vals, csr
