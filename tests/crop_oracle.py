"""Oracle evaluation on a tile-aligned crop of a large frame, for the
differentiation-at-scale checks.

Only Gaussians whose tile rectangle meets the crop can change a crop pixel,
so the oracle runs on that subset with the full frame's camera (the EWA
guard band depends on the image size, so the crop is not a smaller view)
and with every tile outside the crop left empty.  The per-tile lists are
independent of each other, so the crop tiles' lists equal the full set's.

Finite differences move one Gaussian: its old and new records differ, every
other record is unchanged.  `CropFD` re-inserts the moved Gaussian into the
sorted lists of the tiles it touches before or after the move, at the
position the (depth bits, id) order gives it, and re-renders only those
tiles with the oracle.  Pixels of other tiles are unchanged, so the
difference of the two losses over the re-rendered tiles is the difference
of the full losses.  `tests/test_crop_oracle.py` checks this against a full
re-sort."""
from __future__ import annotations

import numpy as np

import oracle

TILE = 16


class Crop:
    """Tile-aligned crop [ty0, ty0+nty) x [tx0, tx0+ntx) of a single view."""

    def __init__(self, view, ty0, tx0, nty, ntx):
        self.view = np.asarray(view, np.float64)
        W, H, self.tx, self.ty = oracle.view_dims(self.view)
        self.W, self.H = W, H
        self.ty0, self.tx0, self.nty, self.ntx = ty0, tx0, nty, ntx

    def tile_mask(self):
        m = np.zeros((self.ty, self.tx), bool)
        m[self.ty0:self.ty0 + self.nty, self.tx0:self.tx0 + self.ntx] = True
        return m.reshape(-1)

    def pixel_mask(self):
        m = np.zeros((self.H, self.W), bool)
        m[self.ty0 * TILE:(self.ty0 + self.nty) * TILE,
          self.tx0 * TILE:(self.tx0 + self.ntx) * TILE] = True
        return m

    def meets(self, rect, touched):
        """Gaussians (of view 0) whose tile rectangle meets the crop."""
        r = rect[0]
        return ((touched[0] > 0) & (r[:, 0] < self.tx0 + self.ntx) & (r[:, 2] > self.tx0)
                & (r[:, 1] < self.ty0 + self.nty) & (r[:, 3] > self.ty0))

    def restrict(self, ranges):
        rg = ranges.copy()
        rg[~self.tile_mask()] = 0
        return rg


def densest_crop(view, rect, touched, size=8):
    """The size x size tile window with the most (tile, Gaussian) pairs."""
    W, H, tx, ty = oracle.view_dims(np.asarray(view, np.float64))
    r = rect[0][touched[0] > 0]
    cnt = np.zeros((ty + 1, tx + 1), np.int64)
    np.add.at(cnt, (r[:, 1], r[:, 0]), 1)
    np.add.at(cnt, (r[:, 3], r[:, 0]), -1)
    np.add.at(cnt, (r[:, 1], r[:, 2]), -1)
    np.add.at(cnt, (r[:, 3], r[:, 2]), 1)
    cnt = cnt.cumsum(0).cumsum(1)[:ty, :tx]
    win = np.lib.stride_tricks.sliding_window_view(cnt, (size, size)).sum(axis=(2, 3))
    cy, cx = np.unravel_index(int(np.argmax(win)), win.shape)
    return Crop(view, int(cy), int(cx), size, size), int(win.max())


class CropFD:
    """Loss L = sum(w * image) over the crop, in FP64, for parameter sets that
    differ from a base set in one Gaussian."""

    def __init__(self, params64, crop: Crop, w):
        self.p = np.ascontiguousarray(params64, np.float64)
        self.crop = crop
        self.w = np.asarray(w, np.float64)          # [1, 3, H, W]
        rec, rect, touched = oracle.preprocess_f64(self.p, crop.view)
        self.rec, self.rect, self.touched = rec, rect, touched
        self.dbits = oracle.depth_bits(rec)
        _, vals, ranges = oracle.bin_sort(rect, touched, self.dbits, crop.view)
        self.lists = {}
        for t in np.nonzero(crop.tile_mask())[0]:
            b, e = ranges[t]
            self.lists[int(t)] = vals[b:e].astype(np.int64)
        # blend-decision signature of every crop pixel for the base set
        self.sig0 = oracle.render_fwd(self.rec, crop.view, vals, crop.restrict(ranges),
                                      signature=True, f32=False)["sig"][0]
        self._vals, self._ranges = vals, crop.restrict(ranges)

    def analytic(self):
        """The oracle's FP64 chain rule of L at the FP64 records, in their
        order and with FP64 decisions: the model the central differences
        differentiate."""
        grec = oracle.render_bwd(self.rec, self.crop.view, self._vals, self._ranges, self.w,
                                 f32=False)
        return oracle.preprocess_bwd(self.p, self.crop.view, grec)

    def _tiles_of(self, rect_row, touched_v):
        c = self.crop
        if touched_v <= 0:
            return set()
        x0, y0, x1, y1 = (int(v) for v in rect_row)
        out = set()
        for ty in range(max(y0, c.ty0), min(y1, c.ty0 + c.nty)):
            for tx in range(max(x0, c.tx0), min(x1, c.tx0 + c.ntx)):
                out.add(ty * c.tx + tx)
        return out

    def _render(self, g, rec_g, rect_g, touched_g, dbits_g, tiles):
        """Render `tiles` with Gaussian g's record replaced."""
        rec = self.rec.copy()
        rec[0, g] = rec_g
        vals, ranges = [], np.zeros((self.crop.tx * self.crop.ty, 2), np.int32)
        pos = 0
        inside_new = self._tiles_of(rect_g, touched_g)
        key_g = (np.uint64(dbits_g) << np.uint64(32)) | np.uint64(g)
        for t in sorted(tiles):
            lst = self.lists[t]
            lst = lst[lst != g]
            if t in inside_new:
                keys = (self.dbits[0, lst].astype(np.uint64) << np.uint64(32)) | lst.astype(np.uint64)
                k = int(np.searchsorted(keys, key_g))
                lst = np.concatenate([lst[:k], [g], lst[k:]])
            ranges[t] = (pos, pos + len(lst))
            pos += len(lst)
            vals.append(lst)
        vals = np.concatenate(vals).astype(np.uint32) if vals else np.zeros(0, np.uint32)
        out = oracle.render_fwd(rec, self.crop.view, vals, ranges, signature=True, f32=False)
        pm = self._pixels(tiles)
        L = float((self.w[0] * out["image"][0])[:, pm].sum())
        return L, out["sig"][0][pm], out["image"][0][:, pm]

    def _pixels(self, tiles):
        m = np.zeros(self.crop.tx * self.crop.ty, bool)
        m[list(tiles)] = True
        pm = np.repeat(np.repeat(m.reshape(self.crop.ty, self.crop.tx), TILE, 0), TILE, 1)
        return pm[:self.crop.H, :self.crop.W]

    def moved(self, g, column):
        """FP64 record, tile rect, tile count and depth bits of Gaussian g
        with the given parameter column."""
        q = np.ascontiguousarray(np.asarray(column, np.float64).reshape(-1, 1))
        rec_g, rect_g, touched_g = oracle.preprocess_f64(q, self.crop.view)
        dbits_g = oracle.depth_bits(rec_g)[0, 0]
        return rec_g[0, 0], rect_g[0, 0], touched_g[0, 0], dbits_g

    def fd(self, g, k, h):
        """Central difference of L in parameter k of Gaussian g, and whether
        every blend decision in the crop is the same at +h and -h as at 0."""
        cp = self.p[:, g].copy()
        cp[k] += h
        plus = self.moved(g, cp)
        cm = self.p[:, g].copy()
        cm[k] -= h
        minus = self.moved(g, cm)
        tiles = self._tiles_of(self.rect[0, g], self.touched[0, g])
        for s in (plus, minus):
            tiles |= self._tiles_of(s[1], s[2])
        if not tiles:
            return 0.0, True
        s0 = self.sig0[self._pixels(tiles)]
        Lp, sp, _ = self._render(g, *plus, tiles)
        Lm, sm, _ = self._render(g, *minus, tiles)
        same = np.array_equal(sp, s0) and np.array_equal(sm, s0)
        return (Lp - Lm) / (2.0 * h), same

    def fd_many(self, cands, h, threads=8):
        """fd() over (g, k) candidates in threads (the oracle's calls hold no
        shared state); results in candidate order."""
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=threads) as ex:
            return list(ex.map(lambda c: self.fd(c[0], c[1], h), cands))
