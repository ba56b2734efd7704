// Exhaustive host check of the library's cell geometry (compiled with g++ by
// tests/test_abi_cpu.py). For one frame shape it verifies that
//   1. the cells' decision boxes partition the detectable interior of every
//      level, each pixel going to the cell of its footprint start (x<<o, y<<o);
//   2. every scale-space neighbour read by a decision (8 in-plane pixels, the
//      finer 4x4 block, the coarser 2x2 block) that lies in the detectable
//      interior of its level is inside that level's score box;
//   3. score boxes stay inside the detectable interior, so the ring of every
//      scored pixel is inside the level.
// Prints "ok <max_lds_bytes> <store_capacity>" or the first violation.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_1503_06959_amd/csrc/kpd_geom.h"

using kpd::Box;

static bool inside(const Box& b, int x, int y) { return x >= b.x0 && x < b.x1 && y >= b.y0 && y < b.y1; }

int main(int argc, char** argv)
{
    if (argc != 6) { fprintf(stderr, "usage: W H O Nc Nr\n"); return 2; }
    const int W = atoi(argv[1]), H = atoi(argv[2]), O = atoi(argv[3]), Nc = atoi(argv[4]), Nr = atoi(argv[5]);
    int w[KPD_MAX_OCTAVES], h[KPD_MAX_OCTAVES];
    for (int o = 0; o < O; ++o) { w[o] = W >> o; h[o] = H >> o; }
    const int ncell = Nc * Nr;
    std::vector<Box> dec((size_t)ncell * O), sb((size_t)ncell * O);
    long cap = 0;
    int lds = 0;
    for (int c = 0; c < ncell; ++c) {
        Box r = kpd::cell_rect(c, W, H, Nc, Nr);
        for (int o = 0; o < O; ++o) dec[(size_t)c * O + o] = kpd::decision_box(r, o, w[o], h[o]);
        for (int o = 0; o < O; ++o) {
            sb[(size_t)c * O + o] = kpd::score_box(&dec[(size_t)c * O], o, O, w[o], h[o]);
            cap += kpd::decision_capacity(dec[(size_t)c * O + o]);
            const Box& s = sb[(size_t)c * O + o];
            if (!kpd::box_empty(s) && (s.x0 < 3 || s.y0 < 3 || s.x1 > w[o] - 3 || s.y1 > h[o] - 3)) {
                printf("score box outside interior c=%d o=%d\n", c, o);
                return 1;
            }
        }
        kpd::CellLayout CL;
        kpd::cell_layout(r, O, w, h, &CL);
        lds = kpd::imax(lds, CL.bytes);
        // every neighbour a decision reads lies in its level's score map
        auto padded = [&](int o, int x, int y) {
            const Box& q = CL.qb[o];
            const Box& s = CL.sb[o];
            // the score box lies inside the query box, and the query box inside the level
            if (!kpd::box_empty(s) && (s.x0 < q.x0 || s.x1 > q.x1 || s.y0 < q.y0 || s.y1 > q.y1)) return false;
            if (q.x0 < 0 || q.y0 < 0 || q.x1 > w[o] || q.y1 > h[o]) return false;
            return x >= q.x0 && x < q.x1 && y >= q.y0 && y < q.y1;
        };
        for (int o = 0; o < O; ++o) {
            const Box& d = CL.dec[o];
            if (kpd::box_empty(d)) continue;
            for (int y = d.y0; y < d.y1; ++y)
                for (int x = d.x0; x < d.x1; ++x) {
                    bool okq = true;
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) okq = okq && padded(o, x + dx, y + dy);
                    if (o > 0)
                        for (int yy = 2 * y - 1; yy <= 2 * y + 2; ++yy)
                            for (int xx = 2 * x - 1; xx <= 2 * x + 2; ++xx) okq = okq && padded(o - 1, xx, yy);
                    if (o + 1 < O)
                        for (int yy = (y - 1) >> 1; yy <= (y + 1) >> 1; ++yy)
                            for (int xx = (x - 1) >> 1; xx <= (x + 1) >> 1; ++xx) okq = okq && padded(o + 1, xx, yy);
                    if (!okq) { printf("query outside padded score map c=%d o=%d (%d,%d)\n", c, o, x, y); return 1; }
                }
        }
        for (int o = 0; o < O; ++o) {
            const Box& s = CL.sb[o];
            if (kpd::box_empty(s)) continue;
            // the pixel tile holds the score box plus the ring apron, inside the level
            if (CL.tx0[o] > s.x0 - 3 || CL.tx0[o] + CL.tpitch[o] < s.x1 + 3 || CL.tx0[o] % 4 ||
                CL.tx0[o] < 0 || CL.tx0[o] + CL.tpitch[o] > ((w[o] + 3) & ~3)) {
                printf("tile columns wrong c=%d o=%d\n", c, o);
                return 1;
            }
            // the group scan visits every score pixel exactly once, with the
            // score index the full test decodes, and its dword reads (the
            // group, its two neighbours, rows -3 and +3) stay in the tile
            const int tp = CL.tpitch[o], hs = kpd::box_h(s), ws = kpd::box_w(s);
            std::vector<int> seen((size_t)ws * hs, 0);
            const int lo_col = s.x0 - CL.tx0[o], hi_col = s.x1 - CL.tx0[o];
            const int ngroups = CL.ngx[o] * hs;
            if (CL.ck_start[o + 1] - CL.ck_start[o] != (ngroups + 63) / 64) {
                printf("group chunks wrong c=%d o=%d\n", c, o);
                return 1;
            }
            for (int g = 0; g < ngroups; ++g) {
                const int ry = (int)(((uint64_t)g * CL.gcm[o]) >> 32);
                if (ry != g / CL.ngx[o]) { printf("group magic wrong c=%d o=%d\n", c, o); return 1; }
                const int cx = 4 * (CL.gx0[o] + g - ry * CL.ngx[o]);
                const long P = (long)(ry + 3) * tp + cx;   // relative to the tile start
                if (P - 4 < 0 || P + 8 > (long)tp * CL.th[o] || P - 3L * tp < 0 || P + 3L * tp + 4 > (long)tp * CL.th[o]) {
                    printf("group read outside the tile c=%d o=%d g=%d\n", c, o, g);
                    return 1;
                }
                for (int k = 0; k < 4; ++k) {
                    if (cx + k < lo_col || cx + k >= hi_col) continue;
                    const int idx = ry * ws + (cx + k - lo_col);
                    if (idx < 0 || idx >= ws * hs) { printf("group index out of range c=%d o=%d\n", c, o); return 1; }
                    ++seen[idx];
                }
            }
            for (int v : seen)
                if (v != 1) { printf("group scan misses or repeats a score pixel c=%d o=%d\n", c, o); return 1; }
        }
    }
    auto interior = [&](int o, int x, int y) { return x >= 3 && y >= 3 && x < w[o] - 3 && y < h[o] - 3; };
    for (int o = 0; o < O; ++o) {
        for (int y = 3; y < h[o] - 3; ++y) {
            for (int x = 3; x < w[o] - 3; ++x) {
                const long X = (long)x << o, Y = (long)y << o;
                const int owner = (int)((Y * Nr) / H) * Nc + (int)((X * Nc) / W);
                int hits = 0;
                for (int c = 0; c < ncell; ++c)
                    if (inside(dec[(size_t)c * O + o], x, y)) {
                        ++hits;
                        if (c != owner) { printf("pixel o=%d (%d,%d) in cell %d, owner %d\n", o, x, y, c, owner); return 1; }
                    }
                if (hits != 1) { printf("pixel o=%d (%d,%d) in %d decision boxes\n", o, x, y, hits); return 1; }
                const Box* S = &sb[(size_t)owner * O];
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx)
                        if (interior(o, x + dx, y + dy) && !inside(S[o], x + dx, y + dy)) {
                            printf("in-plane neighbour missing o=%d (%d,%d)\n", o, x, y);
                            return 1;
                        }
                if (o > 0)
                    for (int yy = 2 * y - 1; yy <= 2 * y + 2; ++yy)
                        for (int xx = 2 * x - 1; xx <= 2 * x + 2; ++xx)
                            if (interior(o - 1, xx, yy) && !inside(S[o - 1], xx, yy)) {
                                printf("finer neighbour missing o=%d (%d,%d)\n", o, x, y);
                                return 1;
                            }
                if (o + 1 < O)
                    for (int YY = kpd::imax(0, y / 2 - 2); YY <= kpd::imin(h[o + 1] - 1, y / 2 + 2); ++YY) {
                        if (!(2 * YY - 1 <= y && y <= 2 * YY + 2)) continue;
                        for (int XX = kpd::imax(0, x / 2 - 2); XX <= kpd::imin(w[o + 1] - 1, x / 2 + 2); ++XX) {
                            if (!(2 * XX - 1 <= x && x <= 2 * XX + 2)) continue;
                            if (interior(o + 1, XX, YY) && !inside(S[o + 1], XX, YY)) {
                                printf("coarser neighbour missing o=%d (%d,%d)\n", o, x, y);
                                return 1;
                            }
                        }
                    }
            }
        }
    }
    printf("ok %d %ld\n", lds, cap);
    return 0;
}
