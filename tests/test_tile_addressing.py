"""Address replay of the batched kernel's tile products (CPU only).

The persistent tile kernel streams each tile with three routines whose full
steps load without bounds checks: rows or columns past the active width are
read at the last valid one and zeroed by a select, and the prologue of each
load ring clamps its step index to the last full step.  These tests replay
the index arithmetic of those routines exactly as the kernel source writes
it (the same ring schedule, lane decomposition, clamps and masks) for every
call the per-tile routine makes, over the tile shapes of the batched parity
test and of the 1024-tile benchmark set at each block width the autotuner
may choose, with every basis width the rank loop can reach, and check every
element touched against its buffer: the tile itself (rows < h, columns < w,
leading dimension lda = w, the tightest case), the scratch slot's regions
(test-matrix rows, block, basis, C^T) and the LDS arena's regions (W, Gram,
fold buffer).  The column product is replayed in both the form the kernel
ships and the rewritten form with unconditional clamped loads that an
earlier inlined build used.  Constants are read from the kernel header.
"""
import math
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2506_22713_amd", "csrc", "eodabe_tiles.hpp")


def _const(name):
    m = re.search(r"constexpr int %s = (\d+);" % name, open(HDR).read())
    assert m, name
    return int(m.group(1))


TILE_MAX, TILE_RMAX, TILE_BMAX = _const("TILE_MAX"), _const("TILE_RMAX"), _const("TILE_BMAX")
TILE_QW = TILE_RMAX + TILE_BMAX
LD = TILE_MAX
# scratch slot (floats), as TileSlot lays it out
SLOT = {}
_off = 0
for _name, _size in (("Om", TILE_BMAX * LD), ("Y", LD * TILE_BMAX), ("Q", LD * TILE_QW),
                     ("CT", LD * TILE_RMAX), ("VP", LD * TILE_RMAX)):
    SLOT[_name] = (_off, _off + _size)
    _off += _size
# LDS arena (doubles) of the basis phase
SMALL64 = 64 * 65
LDS = {"W": (0, TILE_QW * TILE_BMAX), "Gs": (0, SMALL64),
       "fold": (TILE_QW * TILE_BMAX, TILE_QW * TILE_BMAX + 16 * 256)}


def rup(x, a):
    return (x + a - 1) // a * a


def chol_width(f):
    return 16 if f <= 16 else (32 if f <= 32 else 64)


def ring_steps(nfull, pf):
    """Step indices a pf-deep register ring loads (prologue clamped to the
    last full step, then the steady state and its drain), as in the kernel."""
    if nfull <= 0:
        return []
    out = [min(q, nfull - 1) for q in range(pf)]
    c = 0
    while c + 2 * pf <= nfull:
        out += [c + q + pf for q in range(pf)]
        c += pf
    out += [c + q + pf for q in range(pf) if c + q < nfull and c + q + pf < nfull]
    return out


class Mem:
    """Bounds checks for the buffers one tile touches."""

    def __init__(self, h, w):
        self.h, self.w = h, w
        self.count = 0

    def tile(self, rows, cols):
        rows, cols = np.asarray(rows), np.asarray(cols)
        if rows.size == 0 or cols.size == 0:
            return
        self.count += rows.size * cols.size
        assert rows.min() >= 0 and rows.max() < self.h, ("tile rows", rows.min(), rows.max(), self.h)
        assert cols.min() >= 0 and cols.max() < self.w, ("tile cols", cols.min(), cols.max(), self.w)

    @staticmethod
    def region(table, name, base, rows, ld, cols, row_len):
        """Elements base + row * ld + col with col < row_len <= ld inside region `name`."""
        rows, cols = np.asarray(rows), np.asarray(cols)
        if rows.size == 0 or cols.size == 0:
            return
        lo, hi = table[name]
        assert cols.min() >= 0 and cols.max() < row_len <= ld, (name, cols.max(), row_len, ld)
        first = base + rows.min() * ld + cols.min()
        last = base + rows.max() * ld + cols.max()
        assert lo <= first and last < hi, (name, first, last, lo, hi)


LANES = np.arange(64)
R16, G4 = LANES & 15, LANES >> 4


def rowprod(mem, m, n, bname, bbase, ldb, nb, yname, ybase, ldy, a_tr=False):
    """tile_rowprod_t: Y (m x nb, column-major ldy) = A B^T; A m x n
    (the tile, or its transpose view when a_tr), B rows of length n at
    bbase + row * ldb."""
    ctr = max((nb + 15) // 16, 1)
    nfull = n // 16
    steps = np.array(ring_steps(nfull, 4), dtype=np.int64)
    brow = np.array([16 * u + r if 16 * u + r < nb else max(nb - 1, 0) for u in range(ctr) for r in range(16)])
    bcols = (4 * G4[:, None] + 16 * steps[None, :]).ravel() if steps.size else np.zeros(0, np.int64)
    bcols = (bcols[:, None] + np.arange(4)[None, :]).ravel()
    tail = np.zeros(0, np.int64)
    if 16 * nfull < n:
        k = 16 * nfull
        t = (k + 4 * G4[:, None] + np.arange(4)[None, :]).ravel()
        tail = t[t < n]
    for wv in range(4):
        for p0 in range(wv * 64, m, 256):
            rows = p0 + 16 * np.arange(4)[:, None] + R16[None, :]
            rows = np.where(rows < m, rows, m - 1).ravel()
            for cols in (bcols, tail):
                if a_tr:
                    mem.tile(cols, rows)
                else:
                    mem.tile(rows, cols)
            Mem.region(SLOT, bname, bbase, brow, ldb, bcols, n)
            Mem.region(SLOT, bname, bbase, brow, ldb, tail, n)
            # stores: columns < nb, rows < m
            wr = p0 + 16 * np.arange(4)[:, None] + 4 * G4[None, :]
            wr = (wr.ravel()[:, None] + np.arange(4)[None, :]).ravel()
            wr = wr[wr < m]
            Mem.region(SLOT, yname, ybase, np.arange(nb), ldy, wr, m)


def colprod_guarded(mem, m, n, qname, qbase, ldq, r, cname, cbase, ldc, a_tr=False):
    """tile_colprod as shipped: every load guarded by its row / column test."""
    nsteps = (m + 15) // 16
    tr_ = (r + 15) // 16
    for wv in range(4):
        for c0 in range(64 * wv, n, 256):
            kr = (16 * np.arange(nsteps)[:, None] + 4 * G4[None, :]).ravel()
            rows = (kr[:, None] + np.arange(4)[None, :]).ravel()
            rows = rows[rows < m]
            qc = np.array([16 * t + rr for t in range(tr_) for rr in range(16) if 16 * t + rr < r])
            Mem.region(SLOT, qname, qbase, qc, ldq, rows, m)
            ac = c0 + 16 * np.arange(4)[:, None] + R16[None, :]
            ac = ac.ravel()
            ac = ac[ac < n]
            if a_tr:
                mem.tile(ac, rows)
            else:
                mem.tile(rows, ac)
            ii = np.array([i for i in range(16 * tr_) if i < r])
            Mem.region(SLOT, cname, cbase, ii, ldc, ac, n)


def colprod_clamped(mem, m, n, qname, qbase, ldq, r, cname, cbase, ldc, a_tr=False):
    """The rewritten column product of the earlier inlined build: full steps
    load Q at clamped columns and A at clamped columns without guards."""
    tr_ = max((r + 15) // 16, 1)
    nfull = m // 16
    steps = np.array(ring_steps(nfull, 3), dtype=np.int64)
    qcol = np.array([16 * t + rr if 16 * t + rr < r else max(r - 1, 0) for t in range(tr_) for rr in range(16)])
    for wv in range(4):
        for c0 in range(64 * wv, n, 256):
            acl = c0 + 16 * np.arange(4)[:, None] + R16[None, :]
            acl = np.where(acl < n, acl, n - 1).ravel()
            if steps.size:
                qrows = (4 * G4[:, None] + 16 * steps[None, :]).ravel()
                qrows = (qrows[:, None] + np.arange(4)[None, :]).ravel()
                Mem.region(SLOT, qname, qbase, qcol, ldq, qrows, m)
                if a_tr:
                    mem.tile(acl, qrows)
                else:
                    mem.tile(qrows, acl)
            if 16 * nfull < m:
                kr = (16 * nfull + 4 * G4[:, None] + np.arange(4)[None, :]).ravel()
                kr = kr[kr < m]
                Mem.region(SLOT, qname, qbase, qcol, ldq, kr, m)
                if a_tr:
                    mem.tile(acl, kr)
                else:
                    mem.tile(kr, acl)


def xty(m, xname, xbase, ldx, wx, yname, ybase, ldy, wy, oname, obase, ldo):
    """tile_xty_t: out (wx x wy, row-major ldo, in LDS) = X^T Y, X and Y
    column-major in the slot; partial tiles folded through the fold buffer."""
    tx, ty = max((wx + 15) // 16, 1), max((wy + 15) // 16, 1)
    xcol = np.array([16 * t + r if 16 * t + r < wx else max(wx - 1, 0) for t in range(tx) for r in range(16)])
    ycol = np.array([16 * u + r if 16 * u + r < wy else max(wy - 1, 0) for u in range(ty) for r in range(16)])
    for wv in range(4):
        nfull = (m - 16 * wv - 16) // 64 + 1 if m >= 16 * wv + 16 else 0
        steps = np.array(ring_steps(nfull, 2), dtype=np.int64)
        rows = np.zeros(0, np.int64)
        if steps.size:
            k = 16 * wv + 64 * steps
            rows = ((k[:, None] + 4 * G4[None, :]).ravel()[:, None] + np.arange(4)[None, :]).ravel()
        k = 16 * wv + 64 * nfull
        if k < m:
            t = ((k + 4 * G4)[:, None] + np.arange(4)[None, :]).ravel()
            rows = np.concatenate([rows, t[t < m]])
        Mem.region(SLOT, xname, xbase, xcol, ldx, rows, m)
        Mem.region(SLOT, yname, ybase, ycol, ldy, rows, m)
    red = np.arange(tx * ty * 256) + LDS["fold"][0]
    assert red.max() < LDS["fold"][1]
    i = np.arange(wx)
    j = np.arange(wy)
    Mem.region(LDS, oname, obase, i, ldo, j, ldo)


def replay_tile(h, w, b, ranks, clamped_colprod=False):
    """Every product call of the per-tile routine for tile h x w at block
    width b, the basis growing by whole blocks (the widest it can get), and
    the closing C^T for each final rank in `ranks`."""
    mem = Mem(h, w)
    colprod = colprod_clamped if clamped_colprod else colprod_guarded
    tr = h < w
    m, n = (w, h) if tr else (h, w)
    ldk = rup(n, 4)
    om, yb, q0s, ct = SLOT["Om"][0], SLOT["Y"][0], SLOT["Q"][0], SLOT["CT"][0]
    wcols = 0
    for col0 in range(0, n, b):
        f = min(b, n - col0)
        fpad = rup(f, 16)
        Mem.region(SLOT, "Om", om, np.arange(fpad), ldk, np.arange(ldk), ldk)       # tile_omega
        if tr:
            colprod(mem, n, m, "Om", om, ldk, f, "Y", yb, LD, a_tr=False)
        else:
            rowprod(mem, m, n, "Om", om, ldk, f, "Y", yb, LD)
        for _ in range(2):
            for q0 in range(0, wcols, 64):
                wq = min(64, wcols - q0)
                xty(m, "Q", q0s + q0 * LD, LD, wq, "Y", yb, LD, f, "W", q0 * TILE_BMAX, TILE_BMAX)
            xty(m, "Y", yb, LD, f, "Y", yb, LD, f, "Gs", 0, chol_width(f) + 1)
        # append: columns wcols .. wcols + f - 1 of Q
        Mem.region(SLOT, "Q", q0s, np.arange(wcols, wcols + f), LD, np.arange(m), m)
        wcols += f
        if col0 + f >= n or wcols > TILE_RMAX:
            break
    for r in ranks:
        if r < 1 or r > min(wcols, TILE_RMAX):
            continue
        for c0 in range(0, r, 64):
            rc = min(64, r - c0)
            if not tr:
                colprod(mem, m, n, "Q", q0s + c0 * LD, LD, rc, "CT", ct + c0 * LD, LD)
            else:
                rowprod(mem, n, m, "Q", q0s + c0 * LD, LD, rc, "CT", ct + c0 * LD, LD, a_tr=False)
        if r <= 64:
            xty(n, "CT", ct, LD, r, "CT", ct, LD, r, "Gs", 0, chol_width(r) + 1)
    return mem.count


def _parity_shapes():
    shapes = [(h, w) for h, w, _ in W.tile_shapes(5, count=22, lo=64, hi=1024, rank_lo=5, rank_hi=80)]
    return shapes + [(90, 700), (64, 80), (70, 66), (150, 403), (517, 260), (300, 190)]


EDGE_RANKS = [1, 15, 16, 17, 31, 32, 33, 63, 64, 65, 100, 127, 128]


@pytest.mark.parametrize("b", [16, 32, 64])
@pytest.mark.parametrize("clamped", [False, True], ids=["shipped", "clamped_colprod"])
def test_parity_set_tiles_stay_in_bounds(b, clamped):
    total = 0
    for h, w in _parity_shapes():
        total += replay_tile(h, w, b, EDGE_RANKS + [min(h, w)], clamped_colprod=clamped)
    assert total > 0


@pytest.mark.parametrize("part", range(4))
def test_benchmark_tiles_stay_in_bounds(part):
    shapes = W.tile_shapes(0, count=1024)
    for h, w, rho in shapes[part::4]:
        for b in (16, 32, 64):
            replay_tile(h, w, b, [rho, 64, TILE_RMAX], clamped_colprod=(b == 32))


def test_ring_schedule_covers_each_step_once():
    # the ring loads every full step, and only the prologue's clamped
    # indices repeat (the last full step, never computed twice)
    for nfull in range(0, 40):
        for pf in (2, 3, 4):
            s = ring_steps(nfull, pf)
            assert sorted(set(s)) == list(range(nfull))
            extra = len(s) - nfull
            assert extra == (max(pf - nfull, 0) if nfull > 0 else 0)


def test_planted_unclamped_ring_is_caught():
    # a ring without the prologue clamp reads past the last full step of a
    # short row; the replay must flag it
    mem = Mem(64, 20)
    nfull = 20 // 16
    steps = np.arange(4)                                 # unclamped prologue
    cols = ((4 * G4[:, None] + 16 * steps[None, :]).ravel()[:, None] + np.arange(4)).ravel()
    with pytest.raises(AssertionError):
        mem.tile(np.arange(16), cols)
    assert nfull == 1 and math.isfinite(nfull)
