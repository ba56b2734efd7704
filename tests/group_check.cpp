// Exhaustive host check of the group detector's layouts (compiled with g++
// by tests/test_abi_cpu.py). For one frame shape and group shape it walks
// every group the way the kernel does and verifies that
//   1. the group's decision box on each level is the union of its cells'
//      decision boxes, which partition it, each cell's box computed from the
//      level-0 starts of its column and row as the kernel does;
//   2. the 8-pixel score groups cover every pixel of the score box, every
//      scored pixel inside the detectable interior has a place in the score
//      map, queue-entry offsets stay within their bit widths, and the rows
//      the compass pass reads in place (the group's row, not the level's
//      last, and the rows 3 above and below) are level rows, the group
//      starting at or before the last interior column;
//   3. every scale-space neighbour a decision reads (8 in-plane pixels, the
//      finer 4x4 block, the coarser 2x2 block) lies in its level's score map
//      and is either scored or outside the interior (score 0);
//   4. the entry origin is a multiple of 16 and its extent lies in the
//      level's rows;
//   5. LDS regions (bitmaps, score maps, queues) do not overlap, and
//      the bitmap words of each level hold its decision rows.
// Prints "ok <max_lds_bytes> <groups>" or the first violation.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_1503_06959_amd/csrc/kpd_geom.h"

using kpd::Box;

static int fail(const char* what, int g, int o)
{
    printf("%s (group %d, octave %d)\n", what, g, o);
    return 1;
}

int main(int argc, char** argv)
{
    if (argc != 8) { fprintf(stderr, "usage: W H O Nc Nr Gx Gy\n"); return 2; }
    const int W = atoi(argv[1]), H = atoi(argv[2]), O = atoi(argv[3]), Nc = atoi(argv[4]), Nr = atoi(argv[5]);
    const int Gx = atoi(argv[6]), Gy = atoi(argv[7]);
    int w[KPD_MAX_OCTAVES], h[KPD_MAX_OCTAVES];
    for (int o = 0; o < O; ++o) { w[o] = W >> o; h[o] = H >> o; }
    std::vector<int> colx(Nc + 1), rowy(Nr + 1);
    for (int j = 0; j < Nc; ++j) kpd::cell_span(j, Nc, W, &colx[j], &colx[j + 1]);
    for (int j = 0; j < Nr; ++j) kpd::cell_span(j, Nr, H, &rowy[j], &rowy[j + 1]);
    const int ngc = (Nc + Gx - 1) / Gx, ngr = (Nr + Gy - 1) / Gy;
    int lds = 0;
    for (int gr = 0; gr < ngr; ++gr)
        for (int gc = 0; gc < ngc; ++gc) {
            const int g = gr * ngc + gc;
            const int c0 = gc * Gx, c1 = kpd::imin(c0 + Gx, Nc), r0 = gr * Gy, r1 = kpd::imin(r0 + Gy, Nr);
            const Box a = kpd::cell_rect(r0 * Nc + c0, W, H, Nc, Nr);
            const Box b = kpd::cell_rect((r1 - 1) * Nc + c1 - 1, W, H, Nc, Nr);
            kpd::GroupLayout G;
            if (!kpd::group_layout(Box{a.x0, b.x1, a.y0, b.y1}, O, w, h, c0, c1, r0, r1, W, H, Nc, Nr, nullptr, &G))
                return fail("group too large", g, 0);
            const int bytes = kpd::group_lds_bytes(G, kpd::kDetectWaves);
            lds = kpd::imax(lds, bytes);
            // 5) LDS regions in order
            if (G.cand_off != G.nwords * 8) return fail("bitmaps misplaced", g, 0);
            int mprev = 2 * G.nwords * 8;   // end of the previous region
            for (int o = 0; o < O; ++o) {
                const Box q = G.qb[o];
                if (kpd::box_empty(q) || G.vpitch[o] == 0) continue;
                const int mend = G.voff[o] + G.vpitch[o] * kpd::box_h(q) * 2;
                if (G.voff[o] < mprev || mend > G.zero_bytes) return fail("score maps overlap or leave their region", g, o);
                mprev = mend;
            }
            for (int o = 0; o < O; ++o)
                if (G.voff[o] % 16 || G.queue_off % 16 || G.queue_off < G.zero_bytes)
                    return fail("region not 16-byte aligned or queues overlap the maps", g, o);
            // 1) cells partition the group's decision box
            for (int o = 0; o < O; ++o) {
                const Box d = G.dec[o];
                std::vector<int> hit(kpd::box_empty(d) ? 0 : (size_t)kpd::box_w(d) * kpd::box_h(d), 0);
                if (G.ncells != (c1 - c0) * (r1 - r0)) return fail("cell count", g, o);
                for (int k = 0; k < G.ncells; ++k) {
                        const int cx = c0 + k % (c1 - c0), cy = r0 + k / (c1 - c0);
                        if (G.cell_c[k] != cy * Nc + cx) return fail("cell order", g, o);
                        const Box cr = G.cell_rect[k];
                        if (cr.x0 != colx[cx] || cr.x1 != colx[cx + 1] || cr.y0 != rowy[cy] || cr.y1 != rowy[cy + 1])
                            return fail("cell rectangle", g, o);
                        const int x0 = kpd::imax(kpd::shr_ceil(cr.x0, o), 3), x1 = kpd::imin(kpd::shr_ceil(cr.x1, o), w[o] - 3);
                        const int y0 = kpd::imax(kpd::shr_ceil(cr.y0, o), 3), y1 = kpd::imin(kpd::shr_ceil(cr.y1, o), h[o] - 3);
                        const Box ref = kpd::decision_box(kpd::cell_rect(cy * Nc + cx, W, H, Nc, Nr), o, w[o], h[o]);
                        if (x0 < x1 && y0 < y1) {
                            if (ref.x0 != x0 || ref.x1 != x1 || ref.y0 != y0 || ref.y1 != y1)
                                return fail("cell decision box differs from the cell layout's", g, o);
                        } else if (!kpd::box_empty(ref)) {
                            return fail("cell decision box lost", g, o);
                        }
                        for (int y = y0; y < y1; ++y)
                            for (int x = x0; x < x1; ++x) {
                                if (x < d.x0 || x >= d.x1 || y < d.y0 || y >= d.y1) return fail("cell outside the group box", g, o);
                                ++hit[(size_t)(y - d.y0) * kpd::box_w(d) + (x - d.x0)];
                            }
                    }
                for (int v : hit)
                    if (v != 1) return fail("cells do not partition the group box", g, o);
                if (!kpd::box_empty(d)) {
                    if (G.wpr[o] * 64 < kpd::box_w(d)) return fail("bitmap row too short", g, o);
                    if (G.cwoff[o + 1] - G.cwoff[o] != G.wpr[o] * kpd::box_h(d)) return fail("bitmap words wrong", g, o);
                }
            }
            // 2) score groups, map places and tile reads
            std::vector<std::vector<char>> scored(O);
            for (int o = 0; o < O; ++o) {
                scored[o].assign((size_t)w[o] * h[o], 0);
                const int tp = G.tpitch[o], th = G.th[o];
                if (G.nsr[o] == 0) continue;
                if (G.tx0[o] % 16 || tp % 16 || G.ty0[o] < 0 || G.ty0[o] + th > h[o]) return fail("tile placement", g, o);
                if (tp > 2047 || th > 1023) return fail("tile coordinates exceed the queue entries' bits", g, o);
                const long tsz = (long)tp * th;
                const int ngroups = G.ngx[o] * G.nsr[o];
                if (G.ck_start[o + 1] - G.ck_start[o] != (ngroups + 63) / 64) return fail("chunks", g, o);
                for (int gi = 0; gi < ngroups; ++gi) {
                    const int ry = (int)(((uint64_t)gi * G.gcm[o]) >> 32);
                    if (ry != gi / G.ngx[o]) return fail("group magic", g, o);
                    const int row = ry + 3, col = G.gx0[o] + 8 * (gi - ry * G.ngx[o]) - G.tx0[o];
                    const long T = (long)row * tp + col;
                    if (col % 8 || T - 4 < 0 || T + 12 > tsz || T - 3L * tp < 0 || T + 3L * tp + 8 > tsz)
                        return fail("compass read outside the entry extent", g, o);
                    // reads in place: rows 3 above and below the group's row
                    // are level rows, the centre row is not the last, and the
                    // group starts at or before the last interior column
                    const int gxl = G.tx0[o] + col, yl = G.ty0[o] + row;
                    if (yl - 3 < 0 || yl + 3 > h[o] - 1 || yl + 1 > h[o] - 1 || gxl < 0 || gxl > w[o] - 4)
                        return fail("in-place compass read outside the level", g, o);
                    for (int k = 0; k < 8; ++k) {
                        const int x = G.tx0[o] + col + k, y = G.ty0[o] + row;
                        if (x < 3 || x >= w[o] - 3) continue;   // dropped by the full test
                        const long B = (long)(row - 3) * tp + (col + k - 3);
                        if (B < 0 || B + 6L * tp + 6 >= tsz) return fail("full-test window outside the tile", g, o);
                        const Box q = G.qb[o];
                        if (x < G.mx0[o] || x >= G.mx0[o] + G.vpitch[o] || y < q.y0 || y >= q.y1)
                            return fail("scored pixel outside the score map", g, o);
                        scored[o][(size_t)y * w[o] + x] = 1;
                    }
                }
                // the score box is covered
                const Box sb = kpd::score_box(G.dec, o, O, w[o], h[o]);
                for (int y = sb.y0; y < sb.y1; ++y)
                    for (int x = sb.x0; x < sb.x1; ++x)
                        if (!scored[o][(size_t)y * w[o] + x]) return fail("score-box pixel not scored", g, o);
            }
            // 3) suppression reads
            auto readable = [&](int o, int x, int y) {
                const Box q = G.qb[o];
                if (x < G.mx0[o] || x >= G.mx0[o] + G.vpitch[o] || y < q.y0 || y >= q.y1) return false;
                const bool interior = x >= 3 && y >= 3 && x < w[o] - 3 && y < h[o] - 3;
                return !interior || scored[o][(size_t)y * w[o] + x];
            };
            for (int o = 0; o < O; ++o) {
                const Box d = G.dec[o];
                if (kpd::box_empty(d)) continue;
                for (int y = d.y0; y < d.y1; ++y)
                    for (int x = d.x0; x < d.x1; ++x) {
                        bool ok = true;
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dx = -1; dx <= 1; ++dx) ok = ok && readable(o, x + dx, y + dy);
                        if (o > 0)
                            for (int yy = 2 * y - 1; yy <= 2 * y + 2; ++yy)
                                for (int xx = 2 * x - 1; xx <= 2 * x + 2; ++xx) ok = ok && readable(o - 1, xx, yy);
                        if (o + 1 < O)
                            for (int yy = (y - 1) >> 1; yy <= (y + 1) >> 1; ++yy)
                                for (int xx = (x - 1) >> 1; xx <= (x + 1) >> 1; ++xx) ok = ok && readable(o + 1, xx, yy);
                        if (!ok) return fail("suppression read outside the scored map", g, o);
                    }
            }
        }
    printf("ok %d %d\n", lds, ngc * ngr);
    return 0;
}
