// Cell and octave geometry shared by the host library and the kernels.
//
// Coordinates follow the paper's frame I_n of size N_x x N_y (Sec. 3) and its
// N_r x N_c bin grid (Sec. 3.2): level-0 column X lies in cell column
// floor(X * N_c / W), so cell column j spans [ceil(j*W/N_c), ceil((j+1)*W/N_c)).
// A level-o pixel x belongs to the cell of its footprint start x << o, so the
// level-o columns of cell column j are [ceil(X0 / 2^o), ceil(X1 / 2^o)).
#pragma once

#include <stdint.h>

#include "../../include/kpd.h"

#if defined(__HIPCC__)
#define KPD_HD __host__ __device__ inline
#else
#define KPD_HD inline
#endif

namespace kpd {

// Detection keeps 3 pixels away from every level border (the ring radius).
constexpr int kRingR = 3;

struct Box {
    int x0, x1, y0, y1;  // half-open
};

KPD_HD bool box_empty(const Box& b) { return b.x0 >= b.x1 || b.y0 >= b.y1; }
KPD_HD int box_w(const Box& b) { return b.x1 - b.x0; }
KPD_HD int box_h(const Box& b) { return b.y1 - b.y0; }
KPD_HD int imin(int a, int b) { return a < b ? a : b; }
KPD_HD int imax(int a, int b) { return a > b ? a : b; }

KPD_HD int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
KPD_HD int shr_ceil(int a, int o) { return (a + (1 << o) - 1) >> o; }

// Level-0 span [a, b) of cell index j of n along an axis of length len.
KPD_HD void cell_span(int j, int n, int len, int* a, int* b)
{
    *a = ceil_div((int64_t)j * len, n);
    *b = ceil_div((int64_t)(j + 1) * len, n);
}

// Level-0 rectangle of cell c (row-major over grid_cols x grid_rows).
KPD_HD Box cell_rect(int c, int W, int H, int nc, int nr)
{
    Box r;
    cell_span(c % nc, nc, W, &r.x0, &r.x1);
    cell_span(c / nc, nr, H, &r.y0, &r.y1);
    return r;
}

// Pixels of level o (size w_o x h_o) whose keypoint decision belongs to the
// cell with level-0 rectangle r: the cell's level-o columns and rows clipped
// to the detectable interior [3, w_o - 3) x [3, h_o - 3).
KPD_HD Box decision_box(const Box& r, int o, int wo, int ho)
{
    Box d;
    d.x0 = imax(shr_ceil(r.x0, o), kRingR);
    d.x1 = imin(shr_ceil(r.x1, o), wo - kRingR);
    d.y0 = imax(shr_ceil(r.y0, o), kRingR);
    d.y1 = imin(shr_ceil(r.y1, o), ho - kRingR);
    return d;
}

KPD_HD void box_union(Box* acc, bool* have, const Box& b)
{
    if (box_empty(b)) return;
    if (!*have) { *acc = b; *have = true; return; }
    acc->x0 = imin(acc->x0, b.x0); acc->x1 = imax(acc->x1, b.x1);
    acc->y0 = imin(acc->y0, b.y0); acc->y1 = imax(acc->y1, b.y1);
}

// Query region of level o for one cell: every level-o pixel whose score the
// scale-space suppression of the cell's decisions reads. Decisions at level o
// read their 8 in-plane neighbours; decisions at level o+1 read the finer 4x4
// block [2X-1, 2X+2]; decisions at level o-1 read the coarser pixels X with
// 2X-1 <= x <= 2X+2, i.e. [(x-1)>>1, (x+1)>>1]. Every such pixel lies inside
// the level (decisions keep 3 pixels from the border).
KPD_HD Box query_box(const Box* dec, int o, int O)
{
    Box acc = {0, 0, 0, 0};
    bool have = false;
    const Box& d = dec[o];
    if (!box_empty(d)) box_union(&acc, &have, Box{d.x0 - 1, d.x1 + 1, d.y0 - 1, d.y1 + 1});
    if (o + 1 < O && !box_empty(dec[o + 1])) {
        const Box& u = dec[o + 1];
        box_union(&acc, &have, Box{2 * u.x0 - 1, 2 * u.x1 + 1, 2 * u.y0 - 1, 2 * u.y1 + 1});
    }
    if (o > 0 && !box_empty(dec[o - 1])) {
        const Box& f = dec[o - 1];
        box_union(&acc, &have, Box{(f.x0 - 1) >> 1, (f.x1 >> 1) + 1, (f.y0 - 1) >> 1, (f.y1 >> 1) + 1});
    }
    return have ? acc : Box{0, 0, 0, 0};
}

// Score region of level o: the query region clipped to the detectable
// interior [3, w_o - 3) x [3, h_o - 3), outside which every score is 0.
KPD_HD Box score_box(const Box* dec, int o, int O, int wo, int ho)
{
    Box acc = query_box(dec, o, O);
    if (box_empty(acc)) return Box{0, 0, 0, 0};
    acc.x0 = imax(acc.x0, kRingR); acc.x1 = imin(acc.x1, wo - kRingR);
    acc.y0 = imax(acc.y0, kRingR); acc.y1 = imin(acc.y1, ho - kRingR);
    if (box_empty(acc)) return Box{0, 0, 0, 0};
    return acc;
}

// Largest number of keypoints a cell can hold: two keypoints of one level are
// never 8-neighbours, so each 2x2 block of a decision box holds at most one.
KPD_HD int decision_capacity(const Box& d)
{
    if (box_empty(d)) return 0;
    return ((box_w(d) + 1) >> 1) * ((box_h(d) + 1) >> 1);
}

KPD_HD int round_up(int v, int a) { return (v + a - 1) / a * a; }

// Threads per workgroup of the detection kernel and its waves.
constexpr int kDetectBlock = 512;
constexpr int kDetectWaves = kDetectBlock / 64;
// Entries of each wave's private queue of pixels awaiting the full segment
// test: a power of two holding one pass (64 groups of four pixels) on top of
// a part-filled batch of 64.
constexpr int kQueue = 512;

// floor(i / d) = (i * magic) >> 32 for i * d < 2^32, with magic = ceil(2^32 / d)
// kept in 64 bits: the error i * (magic - 2^32/d) / 2^32 < i / 2^32 < 1/d
// cannot carry the quotient past an integer.
KPD_HD uint64_t div_magic(unsigned d) { return (0x100000000ull + d - 1) / d; }

// Everything one detection workgroup needs to know about its cell, computed
// once per stream on the host: the decision and score boxes of every level
// and where each level's pixel tile, score map and the bitmasks live in LDS.
//
// LDS layout (bytes): [keep bitmask: nwords x u64][candidate bitmask: nwords
// x u64][word offsets: nwords x u32][score maps: u16 per level, each over its
// query box, zero outside the score box][pixel tiles: u8 per level][wave
// queues: waves x kQueue x u16]. The queues come last, so a workgroup of
// fewer than kDetectWaves waves needs base_bytes + its waves' queues only. A level's pixel tile covers its score
// box plus the 3-pixel ring apron; its first column is rounded down to a
// multiple of 4 and its row pitch up to one, so that 4-byte aligned rows can
// be loaded a dword at a time. Score pixels are tested in groups of four
// tile columns (one dword of a tile row); groups that cover any score pixel
// of a row are taken 64 at a time, in chunks that never straddle two levels.
struct CellLayout {
    uint64_t ldm[KPD_MAX_OCTAVES];       // div magics: tile dwords per row,
    uint64_t scm[KPD_MAX_OCTAVES];       // score-box width,
    uint64_t dcm[KPD_MAX_OCTAVES];       // decision-box width
    Box dec[KPD_MAX_OCTAVES];
    Box sb[KPD_MAX_OCTAVES];
    Box qb[KPD_MAX_OCTAVES];             // score-map extent (query box)
    int tx0[KPD_MAX_OCTAVES], ty0[KPD_MAX_OCTAVES];   // level coords of tile (0,0)
    int tpitch[KPD_MAX_OCTAVES], th[KPD_MAX_OCTAVES];
    int toff[KPD_MAX_OCTAVES], voff[KPD_MAX_OCTAVES];
    int ld_start[KPD_MAX_OCTAVES + 1];   // flattened dword-load index of each level
    int sc_start[KPD_MAX_OCTAVES + 1];   // flattened score index of each level
    int dc_start[KPD_MAX_OCTAVES + 1];   // flattened decision index of each level
    int ck_start[KPD_MAX_OCTAVES + 1];   // first group chunk (64 groups) of each level
    uint64_t gcm[KPD_MAX_OCTAVES];       // div magic: groups per score row
    int gx0[KPD_MAX_OCTAVES];            // tile dword column of each score row's first group
    int ngx[KPD_MAX_OCTAVES];            // groups (4 tile columns) per score row
    int vpitch[KPD_MAX_OCTAVES];         // score-map row pitch (query-box width)
    int vbytes;                          // bytes of all score maps (zeroed per cell)
    int O;
    int nwords;                          // words of each bitmask
    int cand_off, woff_off, queue_off;
    int base_bytes;                      // bytes before the queues (= queue_off)
    int bytes;                           // with kDetectWaves queues
};

KPD_HD void cell_layout(const Box& rect, int O, const int* w, const int* h, CellLayout* L)
{
    L->O = O;
    for (int o = 0; o < KPD_MAX_OCTAVES; ++o) {
        L->dec[o] = Box{0, 0, 0, 0};
        L->sb[o] = Box{0, 0, 0, 0};
        L->qb[o] = Box{0, 0, 0, 0};
        L->tx0[o] = L->ty0[o] = L->tpitch[o] = L->th[o] = L->toff[o] = L->voff[o] = L->vpitch[o] = 0;
        L->ldm[o] = L->scm[o] = L->dcm[o] = L->gcm[o] = 0;
        L->gx0[o] = L->ngx[o] = 0;
    }
    for (int o = 0; o < O; ++o) L->dec[o] = decision_box(rect, o, w[o], h[o]);
    for (int o = 0; o < O; ++o) L->sb[o] = score_box(L->dec, o, O, w[o], h[o]);
    for (int o = 0; o < O; ++o) L->qb[o] = query_box(L->dec, o, O);
    int nd = 0;
    for (int o = 0; o < O; ++o) {
        L->dc_start[o] = nd;
        if (!box_empty(L->dec[o])) nd += box_w(L->dec[o]) * box_h(L->dec[o]);
    }
    for (int o = O; o <= KPD_MAX_OCTAVES; ++o) L->dc_start[o] = nd;
    L->nwords = (nd + 63) / 64;
    int off = 0;
    off += L->nwords * 8;
    L->cand_off = off;
    off += L->nwords * 8;
    L->woff_off = off;
    off += round_up(L->nwords * 4, 8);
    int sc = 0, ck = 0;
    const int v0 = off;
    for (int o = 0; o < O; ++o) {
        L->voff[o] = off;
        L->sc_start[o] = sc;
        L->vpitch[o] = 0;
        if (!box_empty(L->qb[o])) {
            L->vpitch[o] = box_w(L->qb[o]);
            off += round_up(L->vpitch[o] * box_h(L->qb[o]) * 2, 4);
        }
        if (!box_empty(L->sb[o])) sc += box_w(L->sb[o]) * box_h(L->sb[o]);
    }
    for (int o = O; o <= KPD_MAX_OCTAVES; ++o) L->sc_start[o] = sc;
    L->vbytes = off - v0;
    int ld = 0;
    for (int o = 0; o < O; ++o) {
        L->ld_start[o] = ld;
        L->ck_start[o] = ck;
        L->toff[o] = off;
        L->gx0[o] = L->ngx[o] = 0;
        if (box_empty(L->sb[o])) continue;
        L->tx0[o] = (L->sb[o].x0 - kRingR) & ~3;
        L->ty0[o] = L->sb[o].y0 - kRingR;
        L->tpitch[o] = round_up(L->sb[o].x1 + kRingR - L->tx0[o], 4);
        L->th[o] = box_h(L->sb[o]) + 2 * kRingR;
        L->gx0[o] = (L->sb[o].x0 - L->tx0[o]) >> 2;
        L->ngx[o] = ((L->sb[o].x1 - 1 - L->tx0[o]) >> 2) - L->gx0[o] + 1;
        ck += (L->ngx[o] * box_h(L->sb[o]) + 63) / 64;
        off += L->tpitch[o] * L->th[o];
        ld += (L->tpitch[o] / 4) * L->th[o];
    }
    for (int o = O; o <= KPD_MAX_OCTAVES; ++o) { L->ld_start[o] = ld; L->ck_start[o] = ck; }
    for (int o = 0; o < O; ++o) {
        L->ldm[o] = div_magic(imax(L->tpitch[o] / 4, 1));
        L->scm[o] = div_magic(imax(box_w(L->sb[o]), 1));
        L->dcm[o] = div_magic(imax(box_w(L->dec[o]), 1));
        L->gcm[o] = div_magic(imax(L->ngx[o], 1));
    }
    L->queue_off = round_up(off, 16);
    L->base_bytes = L->queue_off;
    L->bytes = L->queue_off + kDetectWaves * kQueue * 2;
}

// Dynamic LDS of a detection workgroup of `waves` waves for cells whose
// largest layout takes `bytes` (with kDetectWaves queues).
KPD_HD int detect_lds_for(int bytes, int waves) { return bytes - (kDetectWaves - waves) * kQueue * 2; }

// ---------------------------------------------------------------- groups
//
// The group detector covers a rectangle of cells (columns [gc0, gc1), rows
// [gr0, gr1)) with one workgroup. Per octave it keeps one pixel tile and
// one score map for the whole group, so neighbouring cells share their
// aprons, and emits every cell's keypoints in the cell's own (octave, y, x)
// order at the cell's base in a list. On each level the union of the
// cells' decision boxes is the decision box of the group's rectangle,
// because the cells' column and row boundaries map to ceil(X / 2^o).
//
// Score pixels are taken in groups of eight consecutive columns (one lane,
// two dwords of a level row), starting at a multiple of 8: a group may
// cover columns outside the score box, whose scores are computed too and
// land in the score map (which covers them), and columns outside the
// detectable interior, which the full test drops. Pixels are read from the
// levels in place. Queue entries name a pixel by its offset from the
// group's reference corner (tx0, ty0) of each octave: tx0 is a multiple of
// 16 four or more columns left of the first group, ty0 three rows above
// the first score row; tpitch and th bound the offsets.

constexpr int kGroupQueue = 128;     // entries (u32) of each of a wave's two queues
constexpr int kGroupMaxPitch = 2047;  // tile columns fit 11 bits,
constexpr int kGroupMaxRows = 1023;   // tile rows 10 bits (queue entries)
constexpr int kGroupCands = 512;      // candidates of a group listed for suppression
constexpr int kGroupMaxCells = 16;    // cells of one group

struct GroupLayout {
    Box dec[KPD_MAX_OCTAVES];                       // union decision box
    Box qb[KPD_MAX_OCTAVES];                        // query box (what suppression reads)
    int mx0[KPD_MAX_OCTAVES], my0[KPD_MAX_OCTAVES]; // score-map origin (level coords)
    int vpitch[KPD_MAX_OCTAVES];                    // score-map row pitch (u16 elements)
    int voff[KPD_MAX_OCTAVES];                      // score-map LDS byte offset
    int tx0[KPD_MAX_OCTAVES], ty0[KPD_MAX_OCTAVES]; // queue-entry origin (tx0 a multiple of 16, may be < 0)
    int tpitch[KPD_MAX_OCTAVES], th[KPD_MAX_OCTAVES]; // extent of the entries' columns and rows
    int gx0[KPD_MAX_OCTAVES];                       // first 8-px group column (level coords, multiple of 8)
    int ngx[KPD_MAX_OCTAVES];                       // groups per score row
    int sy0[KPD_MAX_OCTAVES], nsr[KPD_MAX_OCTAVES]; // first score row, score rows
    uint64_t gcm[KPD_MAX_OCTAVES];                  // div magic: groups per row
    uint64_t wpm[KPD_MAX_OCTAVES];                  // div magic: bitmap words per row
    int ck_start[KPD_MAX_OCTAVES + 1];              // first 64-group chunk of each octave
    int cwoff[KPD_MAX_OCTAVES + 1];                 // first bitmap word of each octave
    int wpr[KPD_MAX_OCTAVES];                       // bitmap words per decision row
    int w[KPD_MAX_OCTAVES], h[KPD_MAX_OCTAVES];     // level sizes
    int nwords;                                     // words of each bitmap
    int cand_off;                                   // keep bitmap at 0, candidate bitmap here
    int zero_bytes;                                 // bitmaps and score maps: cleared per group
    int queue_off;                                  // wave queues, after the score maps
    int gc0, gc1, gr0, gr1;                         // cells covered
    int O;
    int ncells;                                     // (gc1 - gc0) x (gr1 - gr0), row-major
    // per cell: its index, its first entry in a keypoint list, and its
    // level-0 rectangle (the cell's decision boxes follow from it)
    int cell_c[kGroupMaxCells];
    uint32_t cell_base[kGroupMaxCells];
    Box cell_rect[kGroupMaxCells];
};

// Floor division by 16 for possibly negative values.
KPD_HD int floor16(int v) { return v >= 0 ? (v & ~15) : -((-v + 15) & ~15); }

// Layout of the group of cells [gc0, gc1) x [gr0, gr1) of a frame W x H
// with nc x nr cells, whose level-0 rectangle is r; bases (nullable) gives
// each cell's first entry in a keypoint list. Returns false when the group
// has more than kGroupMaxCells cells or a tile is too large for the 11-bit
// columns and 10-bit rows of the detector's queue entries.
KPD_HD bool group_layout(const Box& r, int O, const int* w, const int* h, int gc0, int gc1, int gr0, int gr1,
                         int W, int H, int nc, int nr, const uint32_t* bases, GroupLayout* G)
{
    G->O = O;
    G->gc0 = gc0; G->gc1 = gc1; G->gr0 = gr0; G->gr1 = gr1;
    G->ncells = (gc1 - gc0) * (gr1 - gr0);
    if (G->ncells > kGroupMaxCells) return false;
    for (int k = 0; k < kGroupMaxCells; ++k) {
        G->cell_c[k] = 0;
        G->cell_base[k] = 0;
        G->cell_rect[k] = Box{0, 0, 0, 0};
        if (k < G->ncells) {
            const int c = (gr0 + k / (gc1 - gc0)) * nc + gc0 + k % (gc1 - gc0);
            G->cell_c[k] = c;
            G->cell_base[k] = bases ? bases[c] : 0u;
            G->cell_rect[k] = cell_rect(c, W, H, nc, nr);
        }
    }
    for (int o = 0; o < KPD_MAX_OCTAVES; ++o) {
        G->dec[o] = G->qb[o] = Box{0, 0, 0, 0};
        G->mx0[o] = G->my0[o] = G->vpitch[o] = G->voff[o] = 0;
        G->tx0[o] = G->ty0[o] = G->tpitch[o] = G->th[o] = 0;
        G->gx0[o] = G->ngx[o] = G->sy0[o] = G->nsr[o] = 0;
        G->gcm[o] = G->wpm[o] = 0;
        G->wpr[o] = 0;
        G->w[o] = o < O ? w[o] : 0;
        G->h[o] = o < O ? h[o] : 0;
    }
    Box dec[KPD_MAX_OCTAVES];
    for (int o = 0; o < O; ++o) dec[o] = decision_box(r, o, w[o], h[o]);
    for (int o = 0; o < O; ++o) {
        G->dec[o] = box_empty(dec[o]) ? Box{0, 0, 0, 0} : dec[o];
        G->qb[o] = query_box(dec, o, O);
    }
    // bitmaps: rows of each decision box, whole words per row
    int nw = 0;
    for (int o = 0; o < O; ++o) {
        G->cwoff[o] = nw;
        if (box_empty(G->dec[o])) continue;
        G->wpr[o] = (box_w(G->dec[o]) + 63) / 64;
        nw += G->wpr[o] * box_h(G->dec[o]);
    }
    for (int o = O; o <= KPD_MAX_OCTAVES; ++o) G->cwoff[o] = nw;
    G->nwords = nw;
    int off = 0;
    off += nw * 8;
    G->cand_off = off;
    off += nw * 8;
    off = round_up(off, 16);
    // score groups and maps
    int ck = 0;
    for (int o = 0; o < O; ++o) {
        G->ck_start[o] = ck;
        const Box sb = score_box(dec, o, O, w[o], h[o]);
        const Box q = G->qb[o];
        if (box_empty(q)) continue;
        int mx0 = q.x0, mx1 = q.x1;
        if (!box_empty(sb)) {
            G->gx0[o] = sb.x0 & ~7;
            G->ngx[o] = ((sb.x1 + 7) & ~7) / 8 - G->gx0[o] / 8;
            G->sy0[o] = sb.y0;
            G->nsr[o] = box_h(sb);
            const int sx0 = imax(G->gx0[o], kRingR), sx1 = imin(G->gx0[o] + 8 * G->ngx[o], w[o] - kRingR);
            mx0 = imin(mx0, sx0);
            mx1 = imax(mx1, sx1);
            ck += (G->ngx[o] * G->nsr[o] + 63) / 64;
        }
        G->mx0[o] = mx0;
        G->my0[o] = q.y0;
        G->vpitch[o] = mx1 - mx0;
        G->voff[o] = off;
        off += round_up(G->vpitch[o] * box_h(q) * 2, 16);
    }
    for (int o = O; o <= KPD_MAX_OCTAVES; ++o) G->ck_start[o] = ck;
    G->zero_bytes = off;
    // queue-entry origins and extents
    for (int o = 0; o < O; ++o) {
        if (G->nsr[o] == 0) continue;
        G->tx0[o] = floor16(G->gx0[o] - 4);
        const int tx1 = round_up(G->gx0[o] + 8 * G->ngx[o] + 4, 16);
        G->tpitch[o] = tx1 - G->tx0[o];
        G->ty0[o] = G->sy0[o] - kRingR;
        G->th[o] = G->nsr[o] + 2 * kRingR;
        if (G->tpitch[o] > kGroupMaxPitch || G->th[o] > kGroupMaxRows) return false;
    }
    G->queue_off = round_up(off, 16);
    for (int o = 0; o < O; ++o) {
        G->gcm[o] = div_magic(imax(G->ngx[o], 1));
        G->wpm[o] = div_magic(imax(G->wpr[o], 1));
    }
    return true;
}

// Dynamic LDS of a group workgroup of `waves` waves: two queues a wave,
// then the suppression list (kGroupCands entries and its count).
KPD_HD int group_lds_bytes(const GroupLayout& G, int waves)
{
    return G.queue_off + waves * 2 * kGroupQueue * 4 + kGroupCands * 4 + 16;
}

}  // namespace kpd
