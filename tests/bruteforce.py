"""Definition-literal brute force for tiny images (pure Python, slow).

Written independently of the oracle and structured differently on purpose,
so that a mistake in one of them shows up as a disagreement:
  * the ring is generated with the midpoint circle algorithm and ordered by
    angle, not taken from a table;
  * the contiguous-arc test searches a doubled bit string;
  * scale-space neighbours are defined geometrically, by the Chebyshev
    distance between pixel-footprint centres in level-0 units;
  * cells come from numpy integer arithmetic on coordinate grids.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np


def bresenham_ring(r: int = 3) -> List[Tuple[int, int]]:
    """Radius-r Bresenham (midpoint) circle, ordered clockwise on screen
    (y grows downwards) starting straight up."""
    pts = set()
    x, y, d = 0, r, 1 - r
    while x <= y:
        for sx in (1, -1):
            for sy in (1, -1):
                pts.add((sx * x, sy * y))
                pts.add((sx * y, sy * x))
        if d < 0:
            d += 2 * x + 3
        else:
            d += 2 * (x - y) + 5
            y -= 1
        x += 1
    return sorted(pts, key=lambda p: math.atan2(p[0], -p[1]) % (2 * math.pi))


RING = bresenham_ring(3)


def has_arc(bits: List[bool], n: int = 9) -> bool:
    s = "".join("1" if b else "0" for b in bits)
    return "1" * n in (s + s)


def pyramid(img: np.ndarray, O: int) -> List[np.ndarray]:
    levels = [img.astype(np.int64)]
    for _ in range(1, O):
        p = levels[-1]
        h, w = p.shape[0] // 2, p.shape[1] // 2
        q = p[:2 * h, :2 * w]
        s = q[0::2, 0::2] + q[0::2, 1::2] + q[1::2, 0::2] + q[1::2, 1::2]
        levels.append((s + 2) // 4)
    return [lv.astype(np.uint8) for lv in levels]


def score(level: np.ndarray, x: int, y: int, t: int) -> int:
    h, w = level.shape
    if not (3 <= x < w - 3 and 3 <= y < h - 3):
        return 0
    p = int(level[y, x])
    ring = [int(level[y + dy, x + dx]) for dx, dy in RING]
    bright = [c > p + t for c in ring]
    dark = [c < p - t for c in ring]
    if not (has_arc(bright) or has_arc(dark)):
        return 0
    sb = sum(c - p - t for c in ring if c > p + t)
    sd = sum(p - c - t for c in ring if c < p - t)
    return max(sb, sd)


def footprint_centre(o: int, x: int, y: int) -> Tuple[float, float]:
    s = 2 ** o
    return ((x + 0.5) * s, (y + 0.5) * s)


def are_neighbours(p: Tuple[int, int, int], q: Tuple[int, int, int]) -> bool:
    """p, q = (octave, x, y). Same level: the 8-neighbourhood. Adjacent
    levels: footprint centres within 3/4 of the coarser pixel's size in both
    axes (equivalently, the 4x4 finer block around the coarser pixel)."""
    (op, xp, yp), (oq, xq, yq) = p, q
    if p == q or abs(op - oq) > 1:
        return False
    cp, cq = footprint_centre(*p), footprint_centre(*q)
    dx, dy = abs(cp[0] - cq[0]), abs(cp[1] - cq[1])
    if op == oq:
        s = 2 ** op
        return max(dx, dy) <= s
    s = 2 ** max(op, oq)
    return max(dx, dy) <= 0.75 * s


def precedes(a: Tuple[int, int, int, int], b: Tuple[int, int, int, int]) -> bool:
    """a, b = (V, octave, y, x); True when a ranks above b."""
    return (-a[0], a[1], a[2], a[3]) < (-b[0], b[1], b[2], b[3])


def detect(img: np.ndarray, t: int, O: int) -> List[Tuple[int, int, int, int]]:
    """F(I) as tuples (x, y, octave, V) ordered by octave, y, x."""
    levels = pyramid(img, O)
    cands: Dict[Tuple[int, int, int], int] = {}
    for o, lv in enumerate(levels):
        h, w = lv.shape
        for y in range(h):
            for x in range(w):
                v = score(lv, x, y, t)
                if v > 0:
                    cands[(o, x, y)] = v
    out = []
    for p, v in cands.items():
        beaten = False
        for q, vq in cands.items():
            if are_neighbours(p, q) and precedes((vq, q[0], q[2], q[1]), (v, p[0], p[2], p[1])):
                beaten = True
                break
        if not beaten:
            out.append((p[1], p[2], p[0], v))
    out.sort(key=lambda k: (k[2], k[1], k[0]))
    return out


def cell_grid(W: int, H: int, Nc: int, Nr: int) -> np.ndarray:
    """Cell index of every level-0 pixel, [H, W]."""
    cx = (np.arange(W, dtype=np.int64) * Nc) // W
    cy = (np.arange(H, dtype=np.int64) * Nr) // H
    return cy[:, None] * Nc + cx[None, :]


def kp_cell(k, W: int, H: int, Nc: int, Nr: int) -> int:
    x, y, o = k[0], k[1], k[2]
    X, Y = x * 2 ** o, y * 2 ** o
    return (Y * Nr // H) * Nc + (X * Nc // W)


class Stream:
    """Eq. (1) over a frame sequence, by brute force."""

    def __init__(self, W, H, t, O, Nc, Nr, TI, TH=0xFFFFFFFF, id_mode=0, layer=0):
        self.W, self.H, self.t, self.O, self.Nc, self.Nr = W, H, t, O, Nc, Nr
        self.TI, self.TH = TI, TH
        self.id_mode, self.layer = id_mode, layer
        self.prev = None
        self.K: List[Tuple[int, int, int, int]] = []
        self.force = True
        self.cells = cell_grid(W, H, Nc, Nr)

    def push(self, frame: np.ndarray):
        nc = self.Nc * self.Nr
        if self.force:
            mask = np.ones(nc, bool)
        else:
            diff = np.abs(frame.astype(np.int64) - self.prev.astype(np.int64))
            sad = np.zeros(nc, np.int64)
            np.add.at(sad, self.cells.ravel(), diff.ravel())
            area = np.bincount(self.cells.ravel(), minlength=nc)
            hist = np.zeros(nc, np.int64)
            for k in self.K:
                hist[kp_cell(k, self.W, self.H, self.Nc, self.Nr)] += 1
            mask = (sad > self.TI * area) | (hist >= self.TH)
        F = detect(frame, self.t, self.O)
        cell = lambda k: kp_cell(k, self.W, self.H, self.Nc, self.Nr)
        if self.id_mode in (1, 2) and not self.force:
            # the changed pixels of pyramid layers, each replicated up to level 0
            layers = [self.layer] if self.id_mode == 1 else list(range(self.O))
            pc, pp = pyramid(frame, max(layers) + 1), pyramid(self.prev, max(layers) + 1)
            up = {}
            for l in layers:
                changed = np.abs(pc[l].astype(np.int64) - pp[l].astype(np.int64)) > self.TI
                lh, lw = changed.shape
                ys = np.minimum(np.arange(self.H) >> l, lh - 1)
                xs = np.minimum(np.arange(self.W) >> l, lw - 1)
                up[l] = changed[ys[:, None], xs[None, :]]
            kb = hist >= self.TH

            def marked(k):
                X, Y = k[0] * 2 ** k[2], k[1] * 2 ** k[2]
                l = self.layer if self.id_mode == 1 else k[2]   # one mask, or the feature's own octave's
                return bool(up[l][Y, X]) or bool(kb[cell(k)])

            new = [k for k in F if marked(k)] + [k for k in self.K if not marked(k)]
            touched = np.zeros(nc, bool)
            for u in up.values():
                touched[np.unique(self.cells[u])] = True
            mask = kb | touched
        else:
            new = [k for k in F if mask[cell(k)]] + [k for k in self.K if not mask[cell(k)]]
        new.sort(key=lambda k: (cell(k), k[2], k[1], k[0]))
        self.K = new
        self.mask = mask.astype(np.uint8)
        self.prev = frame.copy()
        self.force = False
        return new


# ------------------------------------------------- descriptors (R13-R15)

_RINGS = ((0.0, 1, 1), (3.0, 10, 1), (5.0, 14, 1), (7.5, 15, 2), (11.0, 20, 2))   # radius, points, box half-size


def _round_away(v: float) -> int:
    return int(math.copysign(math.floor(abs(v) + 0.5), v))


def desc_points(b: int):
    """Pattern points turned to sector b: (dx, dy, half) per point."""
    pts = []
    for R, n, h in _RINGS:
        for k in range(n):
            a = (2.0 * math.pi * k) / n + (2.0 * math.pi * b) / 32
            pts.append((_round_away(R * math.cos(a)), _round_away(R * math.sin(a)), h))
    return pts


def desc_pairs():
    p0 = desc_points(0)
    d2 = lambda a, b: (p0[a][0] - p0[b][0]) ** 2 + (p0[a][1] - p0[b][1]) ** 2
    pairs = [(a, b) for a in range(60) for b in range(a + 1, 60)]
    long_pairs = [(a, b) for a, b in pairs if d2(a, b) >= 169]
    short = sorted(((d2(a, b), a, b) for a, b in pairs if d2(a, b) < 96))[:512]
    return long_pairs, [(a, b) for _, a, b in short]


def describe(level: np.ndarray, x: int, y: int):
    """Sector and descriptor words (8 x uint64) of the keypoint at (x, y)."""
    padded = np.pad(level.astype(np.int64), 2 + 11 + 2, mode="edge")
    off = 2 + 11 + 2

    def values(b):
        out = []
        for dx, dy, h in desc_points(b):
            cx, cy = x + dx + off, y + dy + off
            box = padded[cy - h:cy + h + 1, cx - h:cx + h + 1]
            out.append(int(box.sum()) * (225 // box.size))
        return out

    long_pairs, short_pairs = desc_pairs()
    p0 = desc_points(0)
    V = values(0)
    gx = sum((p0[b][0] - p0[a][0]) * (V[b] - V[a]) for a, b in long_pairs)
    gy = sum((p0[b][1] - p0[a][1]) * (V[b] - V[a]) for a, b in long_pairs)
    U = [(_round_away(1048576.0 * math.cos((2.0 * math.pi * b) / 32)),
          _round_away(1048576.0 * math.sin((2.0 * math.pi * b) / 32))) for b in range(32)]
    sector = 0
    if gx or gy:
        for b in range(32):
            ux, uy = U[b]
            vx, vy = U[(b + 1) % 32]
            if ux * gy - uy * gx >= 0 and vx * gy - vy * gx < 0:
                sector = b
                break
    V = values(sector)
    words = [0] * 8
    for k, (a, b) in enumerate(short_pairs):
        if V[a] > V[b]:
            words[k >> 6] |= 1 << (k & 63)
    return sector, np.array(words, np.uint64)


# --------------------------------------- sub-pixel and sub-scale refinement

def _fit(level: np.ndarray, t: int, cx: int, cy: int):
    """Least-squares quadratic through the 3 x 3 score patch (numpy lstsq),
    its maximum's offsets (clamped to [-1, 1]) and value."""
    pts, vals = [], []
    for j in (-1, 0, 1):
        for i in (-1, 0, 1):
            pts.append((1.0, i, j, i * i, i * j, j * j))
            vals.append(score(level, cx + i, cy + j, t))
    c = np.linalg.lstsq(np.array(pts), np.array(vals, np.float64), rcond=None)[0]
    # decide concavity on the exact integer multiples of the coefficients
    cxx, cxy, cyy = int(round(6 * c[3])), int(round(4 * c[4])), int(round(6 * c[5]))
    D = 16 * cxx * cyy - 9 * cxy * cxy
    if D > 0 and cxx < 0:
        u, v = np.linalg.solve(np.array([[2 * c[3], c[4]], [c[4], 2 * c[5]]]), -np.array([c[1], c[2]]))
        u, v = float(np.clip(u, -1, 1)), float(np.clip(v, -1, 1))
    else:
        u, v = 0.0, 0.0
    m = c[0] + c[1] * u + c[2] * v + c[3] * u * u + c[4] * u * v + c[5] * v * v
    return u, v, float(m)


def refine(levels, t: int, x: int, y: int, o: int):
    """Refined (x, y), log2 scale and score: fits on the finer, own and
    coarser layers, a parabola along log2 scale, linear interpolation."""
    O = len(levels)
    res = {}
    for k, l in ((0, o - 1), (1, o), (2, o + 1)):
        if 0 <= l < O:
            cx, cy = ((2 * x + 1, 2 * y + 1), (x, y), (x >> 1, y >> 1))[k]
            u, v, m = _fit(levels[l], t, cx, cy)
            res[k] = ((cx + 0.5 + u) * 2 ** l, (cy + 0.5 + v) * 2 ** l, m)
    own = res[1]
    lo = res.get(0, (own[0], own[1], 0.0))
    hi = res.get(2, (own[0], own[1], 0.0))
    q = lo[2] - 2 * own[2] + hi[2]
    tt = float(np.clip((lo[2] - hi[2]) / (2 * q), -1, 1)) if q < 0 else 0.0
    score_v = own[2] + 0.5 * (hi[2] - lo[2]) * tt + 0.5 * q * tt * tt
    other = hi if tt >= 0 else lo
    a = abs(tt)
    return np.array([own[0] + a * (other[0] - own[0]), own[1] + a * (other[1] - own[1]), o + tt, score_v])


# ------------------------------------------- temporally coherent detector

def spiral_offsets(R: int):
    """Grid offsets |u|, |v| <= R in spiral order, by sorting on (ring,
    position along the ring's clockwise perimeter from its top-left corner)."""
    def key(uv):
        u, v = uv
        r = max(abs(u), abs(v))
        if r == 0:
            return (0, 0)
        if v == -r and u < r:
            p = u + r                 # top row, left to right
        elif u == r and v < r:
            p = 2 * r + (v + r)       # right column, downwards
        elif v == r and u > -r:
            p = 4 * r + (r - u)       # bottom row, right to left
        else:
            p = 6 * r + (r - v)       # left column, upwards
        return (r, p)
    return sorted(((u, v) for u in range(-R, R + 1) for v in range(-R, R + 1)), key=key)


def quarter_samples(img: np.ndarray, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Bilinear samples at quarter-pixel positions, exact integers."""
    img = img.astype(np.int64)
    x, y, a, b = X // 4, Y // 4, X % 4, Y % 4
    H, W = img.shape
    x1, y1 = np.minimum(x + 1, W - 1), np.minimum(y + 1, H - 1)
    v = ((4 - a) * (4 - b) * img[y, x] + a * (4 - b) * img[y, x1] + (4 - a) * b * img[y1, x] +
         a * b * img[y1, x1] + 8)
    return v >> 4


def _patch(img, X, Y):
    off = 4 * (np.arange(16) - 8)
    return quarter_samples(img, X + off[None, :], Y + off[:, None])


def _usable(W, H, X, Y):
    return X >= 32 and Y >= 32 and X + 28 <= 4 * (W - 2) and Y + 28 <= 4 * (H - 2)


def _search(cur, ref, X, Y, R, scale, t_et):
    H, W = cur.shape
    best = None
    for u, v in spiral_offsets(R):
        cx, cy = X + scale * u, Y + scale * v
        if not _usable(W, H, cx, cy):
            continue
        sad = int(np.abs(_patch(cur, cx, cy) - ref).sum())
        if best is None or sad < best[0]:
            best = (sad, cx, cy)
        if sad < t_et:
            break
    return best


def track_step(prev: np.ndarray, cur: np.ndarray, tracks, t_bm: int, t_et: int):
    """Block-matching propagation of (x4, y4, octave, score, sad) tracks:
    coarse search over 2-pixel steps within 12 pixels, fine search over
    quarter pixels within 1.75 pixels, both in spiral order with early
    termination; a track survives when the fine SAD is below t_bm."""
    H, W = prev.shape
    out = []
    for x4, y4, o, sc, _ in tracks:
        if not _usable(W, H, x4, y4):
            continue
        ref = _patch(prev, x4, y4)
        c = _search(cur, ref, x4, y4, 6, 8, t_et)
        if c is None:
            continue
        f = _search(cur, ref, c[1], c[2], 7, 1, t_et)
        if f[0] < t_bm:
            out.append((f[1], f[2], o, sc, f[0]))
    return out


# ------------------------------------------------ intra-octave layers

def twothirds(img: np.ndarray) -> np.ndarray:
    """1.5x downsampling: every whole 3x3 block to a 2x2 block, each output
    the rounded mean over the 1.5 x 1.5 area it covers."""
    h, w = img.shape
    bh, bw = h // 3, w // 3
    blocks = img[:3 * bh, :3 * bw].astype(np.int64).reshape(bh, 3, bw, 3)
    wt = np.array([[2, 1, 0], [0, 1, 2]], np.int64)
    s = np.einsum("qj,pi,bjai->bqap", wt, wt, blocks)
    return ((s + 4) // 9).reshape(2 * bh, 2 * bw).astype(np.uint8)


def layer_stack(img: np.ndarray, O: int):
    """[(layer, pixel size in level-0 pixels)] in scale order c0, d0, c1, ..."""
    from fractions import Fraction
    cs = pyramid(img, O)
    ds = [twothirds(img)]
    for _ in range(1, O):
        d = ds[-1]
        h, w = d.shape[0] // 2, d.shape[1] // 2
        q = d[:2 * h, :2 * w].astype(np.int64)
        ds.append(((q[0::2, 0::2] + q[0::2, 1::2] + q[1::2, 0::2] + q[1::2, 1::2] + 2) >> 2).astype(np.uint8))
    out = []
    for i in range(O):
        out.append((cs[i], Fraction(2 ** i)))
        out.append((ds[i], Fraction(3, 2) * 2 ** i))
    return out


def detect_layers(img: np.ndarray, t: int, O: int):
    """Detection over octaves and intra-octaves as tuples (x, y, layer, V) by
    layer, y, x: neighbours on the same or adjacent layers are the pixels
    whose closed level-0 footprints intersect."""
    stack = layer_stack(img, O)
    cands = {}
    for l, (lv, s) in enumerate(stack):
        h, w = lv.shape
        for y in range(h):
            for x in range(w):
                v = score(lv, x, y, t)
                if v > 0:
                    cands[(l, x, y)] = v

    def meet(p, q):
        (lp, xp, yp), (lq, xq, yq) = p, q
        if p == q or abs(lp - lq) > 1:
            return False
        sp, sq = stack[lp][1], stack[lq][1]
        return (max(xp * sp, xq * sq) <= min((xp + 1) * sp, (xq + 1) * sq) and
                max(yp * sp, yq * sq) <= min((yp + 1) * sp, (yq + 1) * sq))

    out = []
    for p, v in cands.items():
        if not any(meet(p, q) and precedes((vq, q[0], q[2], q[1]), (v, p[0], p[2], p[1]))
                   for q, vq in cands.items()):
            out.append((p[1], p[2], p[0], v))
    out.sort(key=lambda k: (k[2], k[1], k[0]))
    return out


def refine_layers(stack, t: int, x: int, y: int, l: int):
    """Refinement on the layers of layer_stack: numpy least-squares fits at
    the pixels holding the footprint centre on layers l-1, l, l+1, a
    parabola (numpy.polyfit) through the fit values along log2 scale, its
    clamped vertex, linear interpolation of the positions in log2 scale."""
    import math
    L = len(stack)

    def sigma(m):
        return m // 2 + (math.log2(1.5) if m % 2 else 0.0)

    s_l = stack[l][1]
    res = {}
    for k, m in ((0, l - 1), (1, l), (2, l + 1)):
        if 0 <= m < L:
            s_m = stack[m][1]
            cx, cy = int((x + 0.5) * s_l / s_m), int((y + 0.5) * s_l / s_m)
            u, v, val = _fit(stack[m][0], t, cx, cy)
            res[k] = (float((cx + 0.5 + u) * s_m), float((cy + 0.5 + v) * s_m), val)
    own = res[1]
    pts = [res.get(k, (own[0], own[1], 0.0)) for k in range(3)]
    sg = [sigma(l - 1), sigma(l), sigma(l + 1)]
    c2, c1, c0 = np.polyfit(sg, [p[2] for p in pts], 2)
    s = sg[1]
    if c2 < -1e-12:
        s = float(np.clip(-c1 / (2 * c2), sg[0], sg[2]))
    score_v = c2 * s * s + c1 * s + c0
    if s >= sg[1]:
        f, other = (s - sg[1]) / (sg[2] - sg[1]), pts[2]
    else:
        f, other = (sg[1] - s) / (sg[1] - sg[0]), pts[0]
    return np.array([own[0] + f * (other[0] - own[0]), own[1] + f * (other[1] - own[1]), s, score_v])


class LayerStream(Stream):
    """Eq. (1) over the octave and intra-octave layers: the per-cell mask,
    detection over the layers, a keypoint's cell from its level-0 footprint
    start (layer pixel size times its coordinate, floored)."""

    def _cell(self, k):
        from fractions import Fraction
        x, y, l = k[0], k[1], k[2]
        s = Fraction(2 ** (l // 2)) * (Fraction(3, 2) if l % 2 else 1)
        X, Y = int(x * s), int(y * s)
        return (Y * self.Nr // self.H) * self.Nc + (X * self.Nc // self.W)

    def push(self, frame: np.ndarray):
        nc = self.Nc * self.Nr
        if self.force:
            mask = np.ones(nc, bool)
        else:
            diff = np.abs(frame.astype(np.int64) - self.prev.astype(np.int64))
            sad = np.zeros(nc, np.int64)
            np.add.at(sad, self.cells.ravel(), diff.ravel())
            area = np.bincount(self.cells.ravel(), minlength=nc)
            hist = np.zeros(nc, np.int64)
            for k in self.K:
                hist[self._cell(k)] += 1
            mask = (sad > self.TI * area) | (hist >= self.TH)
        F = detect_layers(frame, self.t, self.O)
        new = [k for k in F if mask[self._cell(k)]] + [k for k in self.K if not mask[self._cell(k)]]
        new.sort(key=lambda k: (self._cell(k), k[2], k[1], k[0]))
        self.K = new
        self.mask = mask.astype(np.uint8)
        self.prev = frame.copy()
        self.force = False
        return new
