/*
 * CPU oracle for masked multi-scale FAST keypoint detection in video
 * (Baroffio, Cesana, Redondi, Tagliasacchi, "Fast keypoint detection in video
 * sequences", arXiv:1503.06959).
 *
 * TEST INFRASTRUCTURE. This file is a plain, slow, scalar, single-threaded
 * statement of what the detection path computes. It exists only to check the
 * GPU library: the test suite, the smoke check and the benchmark's CPU-baseline
 * leg may load it; the library itself never does. It shares no code, header,
 * table or helper with the GPU path.
 *
 * Every function follows the paper's definitions in the paper's order:
 *   Sec. 2     AST segment test on the radius-3 Bresenham circle; scale space
 *              of octaves by downsampling; non-maxima suppression in a 3x3
 *              scale-space neighbourhood keeping local maxima.
 *   Sec. 3     feature set D_n of frame I_n; detection mask M_n; Eq. (1)
 *              propagation of previous-frame features where the mask is 0.
 *   Sec. 3.1   Eq. (2) intensity-difference mask (polarity and granularity
 *              as read below).
 *   Sec. 3.2   Eq. (3) keypoint histogram over the N_r x N_c bin grid,
 *              Eq. (4) threshold T_H.
 *
 * Readings where the paper is silent or inconsistent (kept in one place):
 *   R1  "O octaves" = levels 0..O-1; level o is the 2x2 box mean of level o-1
 *       with round-half-up ((a+b+c+d+2)>>2), dimensions halved by floor.
 *   R2  AST: n = 9 contiguous of the 16 ring pixels, strict inequalities
 *       (brighter than I_p + t, darker than I_p - t).
 *   R3  Corner score (the paper only says "local maxima"): the FAST score
 *       V = max(sum over bright ring pixels of (c - p - t),
 *               sum over dark ring pixels of (p - c - t)) for pixels passing
 *       the segment test, 0 otherwise.
 *   R4  Scale-space neighbourhood of level-o pixel (x,y): its 8 in-plane
 *       neighbours; at level o-1 the pixels (x',y') with 2x-1<=x'<=2x+2 and
 *       2y-1<=y'<=2y+2; at level o+1 the pixels (X,Y) with 2X-1<=x<=2X+2 and
 *       2Y-1<=y<=2Y+2. Ties are broken by a strict total order: higher V
 *       wins, then the finer octave, then the smaller (y,x). A pixel is a
 *       keypoint iff V>0 and no neighbour beats it.
 *   R5  No candidates within 3 pixels of a level's border.
 *   R6  Cells: level-0 pixel (X,Y) lies in cell (floor(X*Nc/W), floor(Y*Nr/H));
 *       a keypoint at (x,y) of level o lies in the cell of (x<<o, y<<o).
 *   R7  Mask (Eq. 2 printed with inverted polarity; the text asks to detect
 *       where the frame changes): a cell is marked when its summed absolute
 *       level-0 difference exceeds T_I times its pixel count (the mean
 *       absolute difference per pixel exceeds T_I), or when the previous
 *       feature set has at least T_H keypoints in it (Eq. 4 uses >=).
 *       The two tests are OR-ed. The first frame, and the frame after a change
 *       of t, mark every cell.
 *   R8  Eq. (1): D_n is the full-frame detection of I_n restricted to marked
 *       cells together with D_{n-1} restricted to unmarked cells, listed by
 *       cell (row-major), then octave, then y, then x.
 *
 * A second mask mode follows Sec. 3.1 literally (one mask for all octaves,
 * option ii, built on a chosen pyramid layer; Sec. 4 uses the top layer):
 *   R9  The pixel (k,l) of layer L is changed when |L_n(k,l) - L_{n-1}(k,l)|
 *       exceeds T_I (Eq. 2 with the polarity of R7). The mask is upsampled to
 *       level 0 by replication: level-0 pixel (X,Y) takes the value of layer
 *       pixel (X >> L, Y >> L), clamped to the layer's last column and row
 *       for the strip that halving by floor leaves uncovered.
 *   R10 Eq. (1) is applied per feature: a feature at level o, (x,y), sits at
 *       level-0 position p = (x<<o, y<<o) (R6); M_n(p) = 1 when p's layer
 *       pixel changed or p's cell has at least T_H features of D_{n-1}
 *       (Eq. 4, per cell as in R7). D_n holds the features of F(I_n) with
 *       M_n(p) = 1 and those of D_{n-1} with M_n(p) = 0, in the order of R8.
 *       The per-cell mask reported is 1 for a cell marked by T_H or holding
 *       any level-0 pixel whose layer pixel changed.
 *   R11 Switching the mask mode or its layer marks every cell of the next
 *       frame, like a change of t.
 * A third mode takes Sec. 3.1's option i, one mask per octave:
 *   R12 The feature at level o, (x,y), is new when |L_{n,o}(x,y) -
 *       L_{n-1,o}(x,y)| exceeds T_I (the mask built on its own layer, so no
 *       upsampling is involved) or its cell passes the T_H test; otherwise
 *       D_{n-1}'s feature there is kept (Eq. 1 per feature, as in R10). The
 *       per-cell mask reported is 1 for a cell marked by T_H or holding a
 *       level-0 pixel that the upsampled mask of any level (R9) sets.
 *
 * Sec. 3 models a feature as position, scale, orientation and a binary
 * descriptor computed on the patch around the keypoint, and Eq. (1) carries
 * whole features; the paper takes both from BRISK and fixes no parameter.
 * With descriptors switched on (orc_set_descriptors):
 *   R13 Pattern: 60 points in pixels of the keypoint's own level: the
 *       centre and rings of (radius, points) (3, 10), (5, 14), (7.5, 15),
 *       (11, 20); point i of a ring of n points sits at angle 2*pi*i/n, its
 *       offset rounded half away from zero. Each point is smoothed by a box
 *       of half-size 1 (centre and the two inner rings) or 2 (outer rings);
 *       V = box sum * 225 / box area, an exact integer. Pixels outside the
 *       level take the nearest edge pixel.
 *   R14 Orientation: G = sum over long pairs (squared distance >= 169
 *       between the unrotated rounded points) of (p_j - p_i)(V_j - V_i),
 *       unweighted; its angle falls in one of 32 equal sectors, found
 *       exactly against the integer boundary vectors round(2^20 (cos, sin)
 *       (2*pi*b/32)); G = 0 takes sector 0.
 *   R15 Descriptor: the pattern turned by 2*pi*b/32 for sector b (offsets
 *       recomputed from the angles and rounded), smoothed again; bit k is
 *       V_a > V_b for the k-th of the 512 shortest pairs (squared distance
 *       of the unrotated points below 96; ordered by that distance, then a,
 *       then b).
 *   R16 Eq. (1) carries a feature whole: only the keypoints that are new in
 *       D_n get a descriptor computed; carried ones keep theirs.
 * With refinement switched on (orc_set_refine), Sec. 2's sub-pixel and
 * sub-scale interpolation, on the octave layers:
 *   R17 On layer l, the 3 x 3 patch P(i, j) of FAST scores (R3; 0 outside the
 *       candidate region) around a centre pixel is fit by a least-squares
 *       quadratic. With integer sums A = P(1,.) - P(-1,.), B = P(.,1) -
 *       P(.,-1), Cx = P(1,.) + P(-1,.) - 2P(0,.), Cy likewise, E = P(1,1) -
 *       P(1,-1) - P(-1,1) + P(-1,-1), K0 = the 5/2/-1 centre stencil, and
 *       D = 16 Cx Cy - 9 E^2: if D > 0 and Cx < 0 the maximum is at
 *       (U/D, V/D), U = -8 Cy A + 6 E B, V = -8 Cx B + 6 E A, each clamped
 *       to [-1, 1]; otherwise at (0, 0). Its value m follows from the fit.
 *   R18 Layers: the keypoint's own (centre = the keypoint), the finer one
 *       (centre (2x+1, 2y+1)) and the coarser one (centre (x>>1, y>>1)),
 *       the pixels holding the keypoint's footprint centre; a missing layer
 *       has m = 0 and the keypoint's own position. A parabola through the
 *       three m along log2 scale gives t in [-1, 1] (0 when not concave), the
 *       score at its vertex, log2 scale o + t, and the position interpolated
 *       linearly between the own layer's maximum and the finer (t < 0) or
 *       coarser (t > 0) one's, in level-0 pixels ((centre + 0.5 + offset) *
 *       2^l). Every step is an IEEE double operation in a stated order, so
 *       any implementation that keeps the order gets the same bits.
 *   R19 Eq. (1) carries refined values with their features.
 *
 * The comparison system of Sec. 4, the temporally coherent detector (block
 * matching of keypoint patches from frame to frame), as read here:
 *   T1  Groups of Delta frames, counted from the first frame (and from a
 *       reset): the first frame of a group takes the full-frame detection
 *       F(I_n) (R1-R5, in the order of R8, every cell marked); every other
 *       frame propagates the previous frame's keypoints by block matching
 *       and detects nothing.
 *   T2  Positions are in quarter pixels of level 0. A level-o keypoint (x,y)
 *       starts at the centre of its level-0 footprint: 4(x << o) + 2(2^o - 1)
 *       (likewise y). Octave and score travel with it.
 *   T3  A sample at quarter-pixel position (X, Y) (X = 4x + a, Y = 4y + b,
 *       0 <= a, b < 4) is the bilinear mix ((4-a)(4-b)I(x,y) + a(4-b)I(x+1,y)
 *       + (4-a)b I(x,y+1) + ab I(x+1,y+1) + 8) >> 4, exact in integers.
 *   T4  The 16 x 16 patch at (X, Y) holds the samples at (X + 4(i-8),
 *       Y + 4(j-8)), i, j = 0..15. A position is usable when every sample
 *       and its right and lower neighbours lie in the frame: X >= 32,
 *       Y >= 32, X + 28 <= 4(W-2), Y + 28 <= 4(H-2).
 *   T5  Matching cost: the SAD between the keypoint's patch in I_{n-1}, at
 *       its position there, and a candidate patch in I_n. A keypoint whose
 *       own patch is not usable is dropped.
 *   T6  Coarse step: candidates at displacements (2u, 2v) pixels, u, v in
 *       -6..6 (the 24 x 24 window at a precision of 2); fine step: around
 *       the coarse winner, displacements (u/4, v/4), u, v in -7..7 (quarter
 *       pixels up to 1.75 away on each side, so the pixels that the step of
 *       2 skipped are reached). Each step visits its grid in spiral order:
 *       ring r = max(|u|, |v|) outwards; ring r starts at (-r, -r) and walks
 *       clockwise (y down): along the top row to the right, down the right
 *       column, left along the bottom row, up the left column. Unusable
 *       candidates are skipped. The step keeps the lowest SAD, the earliest
 *       on ties, and stops at the first candidate whose SAD is below T_ET.
 *   T7  The keypoint moves to the fine winner when its SAD is below T_BM;
 *       otherwise (or with no usable coarse candidate) it is dropped. The
 *       survivors keep the previous frame's order.
 *
 * BRISK's intra-octave layers (Sec. 2: layers between the octaves, the
 * first one made by downsampling the image by 1.5), for full-frame
 * detection of one image:
 *   L1  Layers in scale order c_0, d_0, c_1, d_1, ..., c_{O-1}, d_{O-1}
 *       (layer index 2i for c_i, 2i+1 for d_i). c_i are the octaves (R1).
 *       d_0 takes every 3 x 3 block of c_0 (only whole blocks) to a 2 x 2
 *       block: output (2a+p, 2b+q) = (sum over i, j of w_p(i) w_q(j)
 *       c_0(3a+i, 3b+j) + 4) / 9 (floor), w_0 = (2, 1, 0), w_1 = (0, 1, 2),
 *       the mean over the 1.5 x 1.5 area the output pixel covers, rounded to
 *       nearest; d_{i+1} halves d_i as R1 does. A pixel of c_i covers 2^i
 *       level-0 pixels a side, one of d_i 1.5 * 2^i.
 *   L2  Every layer is scored as R2, R3, R5.
 *   L3  Two pixels of the same layer, or of layers adjacent in the scale
 *       order, are neighbours when their closed level-0 footprints
 *       [x s, (x+1) s] x [y s, (y+1) s] intersect (s the pixel size); on
 *       one layer these are the 8 neighbours and between octaves exactly
 *       the neighbourhood of R4. A pixel with V > 0 is a keypoint when no
 *       neighbour ranks above it (higher V, then the lower layer index, then
 *       the smaller (y, x)). Keypoints are listed by layer, then y, then x.
 *   L4  Refinement on these layers (R17's fits, R18 generalised): for a
 *       keypoint (x, y) on layer l, the layers l-1, l, l+1 are fitted at the
 *       pixel that holds the keypoint's footprint centre, floor((2x+1) S_l /
 *       (2 S_m)) (S in half level-0 pixels; between octaves this is R18's
 *       (2x+1, 2y+1) and (x>>1, y>>1)). Layer m sits at log2 scale
 *       sigma_m = m/2 for octaves, (m-1)/2 + log2(1.5) for intra-octaves
 *       (log2(1.5) taken as the double nearest to it), extended the same way
 *       to a missing layer, which has value 0 and the keypoint's position.
 *       The parabola through (sigma_k, m_k) in Newton form, d1 = (m_1 -
 *       m_0)/(sigma_1 - sigma_0), d2 likewise, a = (d2 - d1)/(sigma_2 -
 *       sigma_0), has its vertex at sigma* = (sigma_0 + sigma_1)/2 -
 *       d1/(2a) when a < 0, clamped to [sigma_0, sigma_2], else sigma_1; the
 *       score is its value there and the position moves from the own
 *       layer's maximum towards the coarser (sigma* > sigma_1) or finer one's
 *       by the fraction of the way in sigma. Every step is a double
 *       operation in a stated order.
 *   L5  The stream over these layers (orc_set_layers): the mask is R7's and
 *       Eq. (1) is R8's with F(I_n) the detection of L1-L3; a keypoint of
 *       layer l at (x, y) lies in the cell of its level-0 footprint start
 *       (floor(x S_l / 2), floor(y S_l / 2)), S_l in half pixels (R6 for
 *       the octaves), for the mask's histogram, for Eq. (1) and for the
 *       order (cell, layer, y, x). Switching it marks every cell of the
 *       next frame; it runs with the per-cell mask only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t x, y, octave, score;
} orc_kp;

/* ---------------------------------------------------------------- pyramid */

/* Level sizes under R1. Returns the total byte count of levels 0..O-1. */
long orc_level_dims(int W, int H, int O, int* ws, int* hs)
{
    long total = 0;
    int w = W, h = H;
    for (int o = 0; o < O; ++o) {
        ws[o] = w;
        hs[o] = h;
        total += (long)w * h;
        w /= 2;
        h /= 2;
    }
    return total;
}

/* Scale space (Sec. 2; Sec. 3.1 "smoothing and half-sampling"): levels
 * 0..O-1 written back to back into `out`, level 0 being the frame itself. */
int orc_pyramid(const uint8_t* img, int W, int H, int O, uint8_t* out)
{
    int ws[32], hs[32];
    if (O < 1 || O > 32) return -1;
    orc_level_dims(W, H, O, ws, hs);
    memcpy(out, img, (size_t)W * H);
    uint8_t* prev = out;
    for (int o = 1; o < O; ++o) {
        uint8_t* cur = prev + (size_t)ws[o - 1] * hs[o - 1];
        for (int y = 0; y < hs[o]; ++y) {
            for (int x = 0; x < ws[o]; ++x) {
                int pw = ws[o - 1];
                int a = prev[(2 * y) * pw + 2 * x];
                int b = prev[(2 * y) * pw + 2 * x + 1];
                int c = prev[(2 * y + 1) * pw + 2 * x];
                int d = prev[(2 * y + 1) * pw + 2 * x + 1];
                cur[y * ws[o] + x] = (uint8_t)((a + b + c + d + 2) >> 2);
            }
        }
        prev = cur;
    }
    return 0;
}

/* ----------------------------------------------------------- segment test */

/* The 16 pixels of the radius-3 Bresenham circle in circular order,
 * starting straight up and going clockwise (Sec. 2). */
static const int RING[16][2] = {
    {0, -3}, {1, -3}, {2, -2}, {3, -1}, {3, 0}, {3, 1}, {2, 2}, {1, 3},
    {0, 3}, {-1, 3}, {-2, 2}, {-3, 1}, {-3, 0}, {-3, -1}, {-2, -2}, {-1, -3},
};

int orc_ring(int k, int* dx, int* dy)
{
    if (k < 0 || k > 15) return -1;
    *dx = RING[k][0];
    *dy = RING[k][1];
    return 0;
}

/* Is there a run of 9 contiguous set bits on the 16-position circle? */
int orc_arc9(unsigned mask)
{
    for (int s = 0; s < 16; ++s) {
        int run = 1;
        for (int j = 0; j < 9; ++j) {
            if (!((mask >> ((s + j) % 16)) & 1u)) { run = 0; break; }
        }
        if (run) return 1;
    }
    return 0;
}

/* Segment test and score (R2, R3, R5) for one pixel of one level. */
static int score_at(const uint8_t* L, int w, int h, int x, int y, int t)
{
    if (x < 3 || y < 3 || x >= w - 3 || y >= h - 3) return 0;
    int p = L[y * w + x];
    unsigned bright = 0, dark = 0;
    int sum_bright = 0, sum_dark = 0;
    for (int k = 0; k < 16; ++k) {
        int c = L[(y + RING[k][1]) * w + (x + RING[k][0])];
        if (c > p + t) { bright |= 1u << k; sum_bright += c - p - t; }
        if (c < p - t) { dark |= 1u << k; sum_dark += p - c - t; }
    }
    if (!orc_arc9(bright) && !orc_arc9(dark)) return 0;
    return sum_bright > sum_dark ? sum_bright : sum_dark;
}

/* Score map V of one level; V = 0 for pixels failing the segment test. */
int orc_score_level(const uint8_t* L, int w, int h, int t, uint16_t* V)
{
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x)
            V[y * w + x] = (uint16_t)score_at(L, w, h, x, y, t);
    return 0;
}

/* --------------------------------------------------- scale-space maxima */

/* q = (oq, xq, yq, vq) beats p = (op, xp, yp, vp) under the total order of R4. */
static int beats(int vq, int oq, int yq, int xq, int vp, int op, int yp, int xp)
{
    if (vq != vp) return vq > vp;
    if (oq != op) return oq < op;
    if (yq != yp) return yq < yp;
    return xq < xp;
}

/* Full-frame detection F(I) (Sec. 2): pyramid, segment test and score on
 * every level, non-maxima suppression in the scale-space neighbourhood.
 * Output order: octave, then y, then x. Returns the count, or -1 when `cap`
 * is too small, or -2 on bad arguments. */
int orc_detect(const uint8_t* img, int W, int H, int t, int O, orc_kp* out, int cap)
{
    int ws[32], hs[32];
    if (O < 1 || O > 32 || W < 1 || H < 1) return -2;
    long total = orc_level_dims(W, H, O, ws, hs);
    uint8_t* pyr = (uint8_t*)malloc((size_t)total);
    uint16_t* V = (uint16_t*)malloc((size_t)total * sizeof(uint16_t));
    long off[33];
    off[0] = 0;
    for (int o = 0; o < O; ++o) off[o + 1] = off[o] + (long)ws[o] * hs[o];
    orc_pyramid(img, W, H, O, pyr);
    for (int o = 0; o < O; ++o)
        orc_score_level(pyr + off[o], ws[o], hs[o], t, V + off[o]);

    int n = 0;
    for (int o = 0; o < O; ++o) {
        for (int y = 0; y < hs[o]; ++y) {
            for (int x = 0; x < ws[o]; ++x) {
                int v = V[off[o] + (long)y * ws[o] + x];
                if (v == 0) continue;
                int keep = 1;
                /* in-plane 8-neighbourhood */
                for (int dy = -1; dy <= 1 && keep; ++dy)
                    for (int dx = -1; dx <= 1 && keep; ++dx) {
                        int qx = x + dx, qy = y + dy;
                        if ((dx == 0 && dy == 0) || qx < 0 || qy < 0 || qx >= ws[o] || qy >= hs[o]) continue;
                        int vq = V[off[o] + (long)qy * ws[o] + qx];
                        if (beats(vq, o, qy, qx, v, o, y, x)) keep = 0;
                    }
                /* finer octave o-1: 2x-1 <= x' <= 2x+2 */
                if (o > 0)
                    for (int qy = 2 * y - 1; qy <= 2 * y + 2 && keep; ++qy)
                        for (int qx = 2 * x - 1; qx <= 2 * x + 2 && keep; ++qx) {
                            if (qx < 0 || qy < 0 || qx >= ws[o - 1] || qy >= hs[o - 1]) continue;
                            int vq = V[off[o - 1] + (long)qy * ws[o - 1] + qx];
                            if (beats(vq, o - 1, qy, qx, v, o, y, x)) keep = 0;
                        }
                /* coarser octave o+1: 2X-1 <= x <= 2X+2 */
                if (o + 1 < O)
                    for (int qy = y / 2 - 2; qy <= y / 2 + 2 && keep; ++qy)
                        for (int qx = x / 2 - 2; qx <= x / 2 + 2 && keep; ++qx) {
                            if (!(2 * qx - 1 <= x && x <= 2 * qx + 2)) continue;
                            if (!(2 * qy - 1 <= y && y <= 2 * qy + 2)) continue;
                            if (qx < 0 || qy < 0 || qx >= ws[o + 1] || qy >= hs[o + 1]) continue;
                            int vq = V[off[o + 1] + (long)qy * ws[o + 1] + qx];
                            if (beats(vq, o + 1, qy, qx, v, o, y, x)) keep = 0;
                        }
                if (!keep) continue;
                if (n >= cap) { free(pyr); free(V); return -1; }
                out[n].x = x;
                out[n].y = y;
                out[n].octave = o;
                out[n].score = v;
                ++n;
            }
        }
    }
    free(pyr);
    free(V);
    return n;
}

/* ------------------------------------------------------------------ cells */

static int cell_col(int X, int W, int Nc) { return (int)(((long)X * Nc) / W); }
static int cell_row(int Y, int H, int Nr) { return (int)(((long)Y * Nr) / H); }

/* F(I_n) restricted to marked cells, computed the way the masked method
 * saves work on a CPU: the keypoints of pixels whose cell (R6) is marked,
 * with every score taken only when the suppression of such a pixel reads
 * it (scores cached per level, -1 = not taken yet). Equal to orc_detect's
 * list filtered by the mask, in the same order. */
static int lazy_score(uint8_t* const* lv, const int* ws, const int* hs, int32_t* const* V, int t, int o, int x, int y)
{
    if (x < 0 || y < 0 || x >= ws[o] || y >= hs[o]) return 0;
    int32_t* v = &V[o][(long)y * ws[o] + x];
    if (*v < 0) *v = score_at(lv[o], ws[o], hs[o], x, y, t);
    return *v;
}

int orc_detect_masked(const uint8_t* img, int W, int H, int t, int O, const uint8_t* mask, int Nc, int Nr,
                      orc_kp* out, int cap)
{
    int ws[32], hs[32];
    if (O < 1 || O > 32 || W < 1 || H < 1) return -2;
    long total = orc_level_dims(W, H, O, ws, hs);
    uint8_t* pyr = (uint8_t*)malloc((size_t)total);
    int32_t* Vall = (int32_t*)malloc((size_t)total * sizeof(int32_t));
    uint8_t* lv[32];
    int32_t* V[32];
    long off = 0;
    for (int o = 0; o < O; ++o) { lv[o] = pyr + off; V[o] = Vall + off; off += (long)ws[o] * hs[o]; }
    orc_pyramid(img, W, H, O, pyr);
    for (long i = 0; i < total; ++i) Vall[i] = -1;
    int n = 0;
    for (int o = 0; o < O; ++o)
        for (int y = 0; y < hs[o]; ++y) {
            const int row = cell_row(y << o, H, Nr);
            for (int x = 0; x < ws[o]; ++x) {
                if (!mask[row * Nc + cell_col(x << o, W, Nc)]) continue;
                const int v = lazy_score(lv, ws, hs, V, t, o, x, y);
                if (v == 0) continue;
                int keep = 1;
                for (int dy = -1; dy <= 1 && keep; ++dy)
                    for (int dx = -1; dx <= 1 && keep; ++dx) {
                        if (dx == 0 && dy == 0) continue;
                        if (beats(lazy_score(lv, ws, hs, V, t, o, x + dx, y + dy), o, y + dy, x + dx, v, o, y, x))
                            keep = 0;
                    }
                if (o > 0)
                    for (int qy = 2 * y - 1; qy <= 2 * y + 2 && keep; ++qy)
                        for (int qx = 2 * x - 1; qx <= 2 * x + 2 && keep; ++qx)
                            if (beats(lazy_score(lv, ws, hs, V, t, o - 1, qx, qy), o - 1, qy, qx, v, o, y, x)) keep = 0;
                if (o + 1 < O)
                    for (int qy = y / 2 - 2; qy <= y / 2 + 2 && keep; ++qy)
                        for (int qx = x / 2 - 2; qx <= x / 2 + 2 && keep; ++qx) {
                            if (!(2 * qx - 1 <= x && x <= 2 * qx + 2) || !(2 * qy - 1 <= y && y <= 2 * qy + 2)) continue;
                            if (beats(lazy_score(lv, ws, hs, V, t, o + 1, qx, qy), o + 1, qy, qx, v, o, y, x)) keep = 0;
                        }
                if (!keep) continue;
                if (n >= cap) { free(pyr); free(Vall); return -1; }
                out[n].x = x;
                out[n].y = y;
                out[n].octave = o;
                out[n].score = v;
                ++n;
            }
        }
    free(pyr);
    free(Vall);
    return n;
}

/* Cell index (row-major) of a keypoint at level o (R6). */
int orc_cell_of(int x, int y, int o, int W, int H, int Nc, int Nr)
{
    int X = x << o, Y = y << o;
    return cell_row(Y, H, Nr) * Nc + cell_col(X, W, Nc);
}

/* ----------------------------------------------------------------- stream */

/* ------------------------------------------------- descriptors (R13-R16) */

#define ORC_NPTS 60
#define ORC_BINS 32
#define ORC_NBITS 512

static const double ORC_PI = 3.14159265358979323846;
static const double RING_R[5] = {0.0, 3.0, 5.0, 7.5, 11.0};
static const int RING_N[5] = {1, 10, 14, 15, 20};
static const int RING_H[5] = {1, 1, 1, 2, 2};

static int d_ready = 0;
static int d_pt[ORC_BINS][ORC_NPTS][2];   /* rounded offsets per sector (R13, R15) */
static int d_half[ORC_NPTS];
static int d_long[ORC_NPTS * ORC_NPTS][2], d_nlong = 0;
static int d_short[ORC_NBITS][2];
static long long d_ux[ORC_BINS], d_uy[ORC_BINS];

static int round_away(double v) { return (int)lround(v); }

static int pair_d2(int a, int b)
{
    const int dx = d_pt[0][a][0] - d_pt[0][b][0], dy = d_pt[0][a][1] - d_pt[0][b][1];
    return dx * dx + dy * dy;
}

static void desc_tables(void)
{
    if (d_ready) return;
    for (int b = 0; b < ORC_BINS; ++b) {
        int i = 0;
        for (int r = 0; r < 5; ++r)
            for (int k = 0; k < RING_N[r]; ++k, ++i) {
                const double a = (2.0 * ORC_PI * k) / RING_N[r] + (2.0 * ORC_PI * b) / ORC_BINS;
                d_pt[b][i][0] = round_away(RING_R[r] * cos(a));
                d_pt[b][i][1] = round_away(RING_R[r] * sin(a));
                d_half[i] = RING_H[r];
            }
        d_ux[b] = llround(1048576.0 * cos((2.0 * ORC_PI * b) / ORC_BINS));
        d_uy[b] = llround(1048576.0 * sin((2.0 * ORC_PI * b) / ORC_BINS));
    }
    /* long pairs in (a, b) order; short pairs: the 512 shortest */
    int ns = 0;
    static int cand[ORC_NPTS * ORC_NPTS][3];
    for (int a = 0; a < ORC_NPTS; ++a)
        for (int b = a + 1; b < ORC_NPTS; ++b) {
            const int d2 = pair_d2(a, b);
            if (d2 >= 169) { d_long[d_nlong][0] = a; d_long[d_nlong][1] = b; ++d_nlong; }
            if (d2 < 96) { cand[ns][0] = d2; cand[ns][1] = a; cand[ns][2] = b; ++ns; }
        }
    /* selection by (d2, a, b): repeated minimum, plain and obviously ordered */
    for (int k = 0; k < ORC_NBITS; ++k) {
        int best = -1;
        for (int q = 0; q < ns; ++q) {
            if (cand[q][0] < 0) continue;
            if (best < 0 || cand[q][0] < cand[best][0] ||
                (cand[q][0] == cand[best][0] && (cand[q][1] < cand[best][1] ||
                                                 (cand[q][1] == cand[best][1] && cand[q][2] < cand[best][2]))))
                best = q;
        }
        d_short[k][0] = cand[best][1];
        d_short[k][1] = cand[best][2];
        cand[best][0] = -1;
    }
    d_ready = 1;
}

/* R13: smoothed value of pattern point i of sector b around (x, y). */
static int point_value(const uint8_t* L, int w, int h, int x, int y, int b, int i)
{
    const int cx = x + d_pt[b][i][0], cy = y + d_pt[b][i][1], r = d_half[i];
    long sum = 0;
    for (int yy = cy - r; yy <= cy + r; ++yy)
        for (int xx = cx - r; xx <= cx + r; ++xx) {
            const int px = xx < 0 ? 0 : (xx > w - 1 ? w - 1 : xx);
            const int py = yy < 0 ? 0 : (yy > h - 1 ? h - 1 : yy);
            sum += L[(size_t)py * w + px];
        }
    const int area = (2 * r + 1) * (2 * r + 1);
    return (int)(sum * (225 / area));
}

/* Rounded offset of pattern point i in sector b (for checking tables). */
int orc_desc_point(int b, int i, int* dx, int* dy)
{
    if (b < 0 || b >= ORC_BINS || i < 0 || i >= ORC_NPTS) return -1;
    desc_tables();
    *dx = d_pt[b][i][0];
    *dy = d_pt[b][i][1];
    return d_half[i];
}

/* R14-R15: sector and 512-bit descriptor of the keypoint at (x, y) of the
 * level image L (w x h). */
int orc_describe(const uint8_t* L, int w, int h, int x, int y, uint64_t* bits)
{
    desc_tables();
    int V[ORC_NPTS];
    for (int i = 0; i < ORC_NPTS; ++i) V[i] = point_value(L, w, h, x, y, 0, i);
    long long gx = 0, gy = 0;
    for (int q = 0; q < d_nlong; ++q) {
        const int a = d_long[q][0], b = d_long[q][1];
        const long long dv = (long long)V[b] - V[a];
        gx += (long long)(d_pt[0][b][0] - d_pt[0][a][0]) * dv;
        gy += (long long)(d_pt[0][b][1] - d_pt[0][a][1]) * dv;
    }
    int bin = 0;
    if (gx != 0 || gy != 0) {
        for (int b = 0; b < ORC_BINS; ++b) {
            const int n = (b + 1) % ORC_BINS;
            const long long c0 = d_ux[b] * gy - d_uy[b] * gx;   /* >= 0: G at or counterclockwise of boundary b */
            const long long c1 = d_ux[n] * gy - d_uy[n] * gx;   /* < 0: G clockwise of boundary b + 1 */
            if (c0 >= 0 && c1 < 0) { bin = b; break; }
        }
    }
    for (int i = 0; i < ORC_NPTS; ++i) V[i] = point_value(L, w, h, x, y, bin, i);
    for (int k = 0; k < ORC_NBITS / 64; ++k) bits[k] = 0;
    for (int k = 0; k < ORC_NBITS; ++k)
        if (V[d_short[k][0]] > V[d_short[k][1]]) bits[k >> 6] |= 1ull << (k & 63);
    return bin;
}

/* ------------------------------------------------------ refinement (R17-R19) */

/* R17: the quadratic fit of the 3 x 3 score patch of layer L around (cx, cy);
 * the maximum's offsets and value. */
static void fit_patch(const uint8_t* L, int w, int h, int t, int cx, int cy, double* u, double* v, double* m)
{
    long P[3][3];   /* P[i + 1][j + 1]: x offset i, y offset j */
    for (int i = -1; i <= 1; ++i)
        for (int j = -1; j <= 1; ++j) P[i + 1][j + 1] = score_at(L, w, h, cx + i, cy + j, t);
    long sx[3], sy[3];
    for (int k = 0; k < 3; ++k) {
        sx[k] = P[k][0] + P[k][1] + P[k][2];
        sy[k] = P[0][k] + P[1][k] + P[2][k];
    }
    const long A = sx[2] - sx[0], B = sy[2] - sy[0];
    const long Cx = sx[2] + sx[0] - 2 * sx[1], Cy = sy[2] + sy[0] - 2 * sy[1];
    const long E = P[2][2] - P[2][0] - P[0][2] + P[0][0];
    const long K0 = -P[0][0] + 2 * P[1][0] - P[2][0] + 2 * P[0][1] + 5 * P[1][1] + 2 * P[2][1] - P[0][2] +
                    2 * P[1][2] - P[2][2];
    const long D = 16 * Cx * Cy - 9 * E * E;
    long U = 0, V = 0, Dn = 1;
    if (D > 0 && Cx < 0) {
        U = -8 * Cy * A + 6 * E * B;
        V = -8 * Cx * B + 6 * E * A;
        Dn = D;
        if (U > D) U = D;
        if (U < -D) U = -D;
        if (V > D) V = D;
        if (V < -D) V = -D;
    }
    *u = (double)U / (double)Dn;
    *v = (double)V / (double)Dn;
    double f = (double)K0 / 9.0;
    f = f + ((double)A / 6.0) * *u;
    f = f + ((double)B / 6.0) * *v;
    f = f + (((double)Cx / 6.0) * *u) * *u;
    f = f + (((double)E / 4.0) * *u) * *v;
    f = f + (((double)Cy / 6.0) * *v) * *v;
    *m = f;
}

/* R18: refined position (level-0 pixels), log2 scale and score of the
 * keypoint (x, y) of level o; lv[l], ws[l], hs[l] are the pyramid levels. */
void orc_refine_kp(uint8_t* const* lv, const int* ws, const int* hs, int O, int t, int x, int y, int o, float* out)
{
    double m[3] = {0.0, 0.0, 0.0}, X[3], Y[3];   /* finer, own, coarser */
    for (int k = 0; k < 3; ++k) {
        const int l = o - 1 + k;
        if (l < 0 || l >= O) continue;
        const int cx = k == 0 ? 2 * x + 1 : (k == 1 ? x : x >> 1);
        const int cy = k == 0 ? 2 * y + 1 : (k == 1 ? y : y >> 1);
        double u, v;
        fit_patch(lv[l], ws[l], hs[l], t, cx, cy, &u, &v, &m[k]);
        X[k] = (((double)cx + 0.5) + u) * (double)(1 << l);
        Y[k] = (((double)cy + 0.5) + v) * (double)(1 << l);
    }
    if (o == 0) { X[0] = X[1]; Y[0] = Y[1]; }
    if (o + 1 >= O) { X[2] = X[1]; Y[2] = Y[1]; }
    const double q = (m[0] - 2.0 * m[1]) + m[2];
    double tt = 0.0;
    if (q < 0.0) {
        tt = (m[0] - m[2]) / (2.0 * q);
        if (tt > 1.0) tt = 1.0;
        if (tt < -1.0) tt = -1.0;
    }
    const double score = (m[1] + (0.5 * (m[2] - m[0])) * tt) + (0.5 * q) * (tt * tt);
    double px, py;
    if (tt >= 0.0) {
        px = X[1] + tt * (X[2] - X[1]);
        py = Y[1] + tt * (Y[2] - Y[1]);
    } else {
        px = X[1] + (-tt) * (X[0] - X[1]);
        py = Y[1] + (-tt) * (Y[0] - Y[1]);
    }
    out[0] = (float)px;
    out[1] = (float)py;
    out[2] = (float)((double)o + tt);
    out[3] = (float)score;
}

typedef struct {
    int W, H, O, Nc, Nr;
    int t;
    int32_t TI;
    uint32_t TH;
    int n_frames;
    int force_all;
    int id_mode;         /* 0: per-cell mean at level 0 (R7); 1: per-pixel on a layer (R9, R10);
                            2: per-pixel on every level, one mask per octave (R12) */
    int id_layer;
    uint8_t* prev;       /* I_{n-1} */
    orc_kp* K;           /* D_{n-1}, then D_n */
    int nK;
    int capK;
    uint8_t* mask;       /* M_n per cell */
    int desc_on;         /* R13-R16: descriptors kept with D_n */
    int ref_on;          /* R17-R19: refined position, scale and score kept with D_n */
    int layers_on;       /* L5: detection over octaves and intra-octaves */
    int lazy;            /* CPU-masked mode: scores only where marked cells' suppression reads them */
    float* ref;          /* 4 floats per feature of D_n */
    uint64_t* desc;      /* 8 words per feature of D_n */
    int32_t* bin;        /* orientation sector per feature of D_n */
    int64_t* sad;        /* per-cell summed |I_n - I_{n-1}| */
    uint32_t* count;     /* per-cell keypoint count of D_n */
} orc_stream;

orc_stream* orc_open(int W, int H, int t, int O, int Nc, int Nr, int32_t TI, uint32_t TH)
{
    if (W < 1 || H < 1 || O < 1 || O > 32 || Nc < 1 || Nr < 1 || Nc > W || Nr > H) return NULL;
    orc_stream* s = (orc_stream*)calloc(1, sizeof(orc_stream));
    s->W = W; s->H = H; s->O = O; s->Nc = Nc; s->Nr = Nr;
    s->t = t; s->TI = TI; s->TH = TH;
    s->prev = (uint8_t*)malloc((size_t)W * H);
    s->capK = W * H + 16;  /* no two keypoints of one level are 8-neighbours */
    s->K = (orc_kp*)malloc(sizeof(orc_kp) * (size_t)s->capK);
    s->mask = (uint8_t*)calloc((size_t)Nc * Nr, 1);
    s->sad = (int64_t*)calloc((size_t)Nc * Nr, sizeof(int64_t));
    s->count = (uint32_t*)calloc((size_t)Nc * Nr, sizeof(uint32_t));
    s->force_all = 1;
    return s;
}

void orc_close(orc_stream* s)
{
    if (!s) return;
    free(s->prev); free(s->K); free(s->mask); free(s->sad); free(s->count); free(s->desc); free(s->bin); free(s->ref);
    free(s);
}

/* A change of t changes every score, so the next frame re-detects every
 * cell; T_I and T_H apply from the next frame on. */
int orc_set_thresholds(orc_stream* s, int t, int32_t TI, uint32_t TH)
{
    if (t != s->t) s->force_all = 1;
    s->t = t; s->TI = TI; s->TH = TH;
    return 0;
}

/* Mask mode from the next frame on: 0 = R7, 1 = R9/R10 on pyramid layer
 * `layer` (0..O-1), 2 = R12 (layer must be 0). A change marks every cell of
 * the next frame (R11). */
int orc_set_id_mode(orc_stream* s, int mode, int layer)
{
    if (mode < 0 || mode > 2 || layer < 0 || layer >= s->O || (mode == 2 && layer != 0)) return -1;
    if (mode == s->id_mode && (mode == 0 || layer == s->id_layer)) return 0;
    s->id_mode = mode;
    s->id_layer = mode == 1 ? layer : 0;
    s->force_all = 1;   /* a new mask re-detects every cell once */
    return 0;
}

/* Keep a descriptor with every feature of D_n (R13-R16) from the next frame
 * on; switching on re-detects every cell once, so that every feature has
 * one. */
/* L5: detection over octaves and intra-octaves from the next frame on
 * (per-cell mask, no descriptors or refinement); a change marks every
 * cell of the next frame */
int orc_set_layers(orc_stream* s, int on)
{
    if (on && (s->desc_on || s->ref_on || s->id_mode != 0)) return -1;
    if ((on != 0) != s->layers_on) s->force_all = 1;
    s->layers_on = on != 0;
    return 0;
}

/* CPU-masked mode (same results): full-frame detection is replaced by
 * detection that scores only what the marked cells' suppression reads */
int orc_set_lazy(orc_stream* s, int on)
{
    s->lazy = on != 0;
    return 0;
}

int orc_set_descriptors(orc_stream* s, int on)
{
    if (on && !s->desc_on) {
        s->desc = (uint64_t*)calloc((size_t)s->capK * 8, sizeof(uint64_t));
        s->bin = (int32_t*)calloc((size_t)s->capK, sizeof(int32_t));
        s->force_all = 1;
    }
    s->desc_on = on != 0;
    return 0;
}

/* Keep the refined position, log2 scale and score with every feature of
 * D_n (R17-R19) from the next frame on; switching on re-detects every cell
 * once. */
int orc_set_refine(orc_stream* s, int on)
{
    if (on && !s->ref_on) {
        s->ref = (float*)calloc((size_t)s->capK * 4, sizeof(float));
        s->force_all = 1;
    }
    s->ref_on = on != 0;
    return 0;
}

/* Copy out the refined values (x, y, log2 scale, score) of D_n. */
int orc_get_refined(orc_stream* s, float* out, int cap)
{
    if (!s->ref_on || cap < s->nK) return -1;
    memcpy(out, s->ref, sizeof(float) * 4 * (size_t)s->nK);
    return s->nK;
}

/* Copy out the descriptors (8 words each) and sectors of D_n. */
int orc_get_desc(orc_stream* s, uint64_t* bits, int32_t* bins, int cap)
{
    if (!s->desc_on || cap < s->nK) return -1;
    memcpy(bits, s->desc, sizeof(uint64_t) * 8 * (size_t)s->nK);
    memcpy(bins, s->bin, sizeof(int32_t) * (size_t)s->nK);
    return s->nK;
}

/* A reset (a scene cut signalled by the caller) treats the next frame like
 * the first one: every cell is detected. */
int orc_reset(orc_stream* s)
{
    s->force_all = 1;
    return 0;
}

static int kp_cmp_ctx_W, kp_cmp_ctx_H, kp_cmp_ctx_Nc, kp_cmp_ctx_Nr, kp_cmp_ctx_layers;

/* Cell of a keypoint: R6, or with layers (L5) the cell of its level-0
 * footprint start, floor(x S_l / 2) with S_l in half pixels */
static int kp_cell(int layers, const orc_kp* k, int W, int H, int Nc, int Nr)
{
    if (!layers) return orc_cell_of(k->x, k->y, k->octave, W, H, Nc, Nr);
    const int l = k->octave, S = l % 2 == 0 ? (2 << (l / 2)) : (3 << (l / 2));
    const int X = (int)(((long)k->x * S) / 2), Y = (int)(((long)k->y * S) / 2);
    return cell_row(Y, H, Nr) * Nc + cell_col(X, W, Nc);
}

int orc_detect_layers(const uint8_t* img, int W, int H, int t, int O, orc_kp* out, int cap);

static int kp_cmp(const void* a, const void* b)
{
    const orc_kp* p = (const orc_kp*)a;
    const orc_kp* q = (const orc_kp*)b;
    int cp = kp_cell(kp_cmp_ctx_layers, p, kp_cmp_ctx_W, kp_cmp_ctx_H, kp_cmp_ctx_Nc, kp_cmp_ctx_Nr);
    int cq = kp_cell(kp_cmp_ctx_layers, q, kp_cmp_ctx_W, kp_cmp_ctx_H, kp_cmp_ctx_Nc, kp_cmp_ctx_Nr);
    if (cp != cq) return cp < cq ? -1 : 1;
    if (p->octave != q->octave) return p->octave < q->octave ? -1 : 1;
    if (p->y != q->y) return p->y < q->y ? -1 : 1;
    if (p->x != q->x) return p->x < q->x ? -1 : 1;
    return 0;
}

typedef struct {
    orc_kp k;
    int32_t bin;
    uint64_t bits[8];
    float ref[4];
} orc_feat;

static int feat_cmp(const void* a, const void* b)
{
    return kp_cmp(&((const orc_feat*)a)->k, &((const orc_feat*)b)->k);
}

/* R10 and R12: M_n for feature k, read on layer id_layer at k's level-0
 * position (mode 1) or on k's own level at (x,y) (mode 2); pix[l], lw[l],
 * lh[l] are layer l's changed pixels and size. The cell mask of s holds the
 * T_H test at this point. */
static int pixel_mask(const orc_stream* s, uint8_t* const* pix, const int* lw, const int* lh, const orc_kp* k)
{
    const int l = s->id_mode == 1 ? s->id_layer : k->octave;
    const int X = k->x << k->octave, Y = k->y << k->octave;
    int kx = X >> l, ly = Y >> l;
    if (kx > lw[l] - 1) kx = lw[l] - 1;
    if (ly > lh[l] - 1) ly = lh[l] - 1;
    if (pix[l][ly * lw[l] + kx]) return 1;
    return s->mask[orc_cell_of(k->x, k->y, k->octave, s->W, s->H, s->Nc, s->Nr)] != 0;
}

/* One frame: detection mask (Eqs. 2-4 as read in R7, or R9/R10), full
 * detection F(I_n), and Eq. (1). */
int orc_push(orc_stream* s, const uint8_t* frame)
{
    const int W = s->W, H = s->H, Nc = s->Nc, Nr = s->Nr;
    const int ncell = Nc * Nr;

    /* detection mask M_n */
    uint8_t* pix[32] = {0};  /* R9: changed pixels of layer l (mode 1: l = id_layer; mode 2: every l) */
    int lw[32] = {0}, lh[32] = {0};
    const int per_pixel = s->id_mode != 0 && !s->force_all;
    const int l0 = s->id_mode == 1 ? s->id_layer : 0, l1 = s->id_mode == 1 ? s->id_layer : s->O - 1;
    if (per_pixel) {
        orc_level_dims(W, H, l1 + 1, lw, lh);
        size_t tot = 0;
        for (int o = 0; o <= l1; ++o) tot += (size_t)lw[o] * lh[o];
        uint8_t* pc = (uint8_t*)malloc(tot);
        uint8_t* pp = (uint8_t*)malloc(tot);
        orc_pyramid(frame, W, H, l1 + 1, pc);
        orc_pyramid(s->prev, W, H, l1 + 1, pp);
        size_t off = 0;
        for (int l = 0; l <= l1; ++l) {
            if (l >= l0) {
                pix[l] = (uint8_t*)malloc((size_t)lw[l] * lh[l]);
                for (int i = 0; i < lw[l] * lh[l]; ++i) {
                    int d = (int)pc[off + i] - (int)pp[off + i];
                    pix[l][i] = (uint8_t)((d < 0 ? -d : d) > s->TI);
                }
            }
            off += (size_t)lw[l] * lh[l];
        }
        free(pc);
        free(pp);
    }
    if (s->force_all) {
        for (int c = 0; c < ncell; ++c) { s->mask[c] = 1; s->sad[c] = 0; }
    } else {
        int64_t* area = (int64_t*)calloc((size_t)ncell, sizeof(int64_t));
        uint32_t* hist = (uint32_t*)calloc((size_t)ncell, sizeof(uint32_t));
        for (int c = 0; c < ncell; ++c) s->sad[c] = 0;
        for (int Y = 0; Y < H; ++Y)
            for (int X = 0; X < W; ++X) {
                int c = cell_row(Y, H, Nr) * Nc + cell_col(X, W, Nc);
                int d = (int)frame[Y * W + X] - (int)s->prev[Y * W + X];
                s->sad[c] += d < 0 ? -d : d;
                area[c] += 1;
            }
        /* Eq. (3): histogram of the previous feature set over the bins */
        for (int i = 0; i < s->nK; ++i)
            hist[kp_cell(s->layers_on, &s->K[i], W, H, Nc, Nr)] += 1;
        for (int c = 0; c < ncell; ++c) {
            int id = s->sad[c] > (int64_t)s->TI * area[c];   /* Eq. (2), R7 */
            int kb = hist[c] >= s->TH;                         /* Eq. (4) */
            s->mask[c] = (uint8_t)(id || kb);
        }
        if (per_pixel) {
            /* R10, R12: the cell mask is the T_H test; the reported mask
             * also flags cells with a changed layer pixel */
            for (int c = 0; c < ncell; ++c) s->mask[c] = (uint8_t)(hist[c] >= s->TH);
            for (int c = 0; c < ncell; ++c) s->sad[c] = 0;
        }
        free(area);
        free(hist);
    }

    /* full-frame detection of I_n */
    orc_kp* F = (orc_kp*)malloc(sizeof(orc_kp) * (size_t)s->capK);
    int nF;
    if (s->layers_on)
        nF = orc_detect_layers(frame, W, H, s->t, s->O, F, s->capK);
    else if (s->lazy && !per_pixel)
        nF = orc_detect_masked(frame, W, H, s->t, s->O, s->mask, Nc, Nr, F, s->capK);
    else
        nF = orc_detect(frame, W, H, s->t, s->O, F, s->capK);
    if (nF < 0) { free(F); return -1; }

    /* Eq. (1): new features where the mask is 1, previous ones elsewhere;
     * with descriptors, new features get theirs computed (R16) */
    orc_feat* D = (orc_feat*)calloc((size_t)(nF + s->nK + 1), sizeof(orc_feat));
    uint8_t* pyr = NULL;
    int dws[32], dhs[32];
    size_t doff[32];
    uint8_t* lvp[32];
    if (s->desc_on || s->ref_on) {
        const long tot = orc_level_dims(W, H, s->O, dws, dhs);
        pyr = (uint8_t*)malloc((size_t)tot);
        orc_pyramid(frame, W, H, s->O, pyr);
        size_t off = 0;
        for (int o = 0; o < s->O; ++o) { doff[o] = off; lvp[o] = pyr + off; off += (size_t)dws[o] * dhs[o]; }
    }
    int nD = 0;
    for (int i = 0; i < nF; ++i) {
        const int keep = per_pixel ? pixel_mask(s, pix, lw, lh, &F[i])
                                   : s->mask[kp_cell(s->layers_on, &F[i], W, H, Nc, Nr)] != 0;
        if (!keep) continue;
        D[nD].k = F[i];
        if (s->desc_on) {
            const int o = F[i].octave;
            D[nD].bin = orc_describe(pyr + doff[o], dws[o], dhs[o], F[i].x, F[i].y, D[nD].bits);
        }
        if (s->ref_on) orc_refine_kp(lvp, dws, dhs, s->O, s->t, F[i].x, F[i].y, F[i].octave, D[nD].ref);
        ++nD;
    }
    /* a forced frame marks every cell and carries nothing (D_{n-1} may come
     * from another scale space after a switch, L5) */
    for (int i = 0; i < (s->force_all ? 0 : s->nK); ++i) {
        const int keep = per_pixel ? !pixel_mask(s, pix, lw, lh, &s->K[i])
                                   : !s->mask[kp_cell(s->layers_on, &s->K[i], W, H, Nc, Nr)];
        if (!keep) continue;
        D[nD].k = s->K[i];
        if (s->desc_on) {
            D[nD].bin = s->bin[i];
            memcpy(D[nD].bits, s->desc + (size_t)i * 8, sizeof(D[nD].bits));
        }
        if (s->ref_on) memcpy(D[nD].ref, s->ref + (size_t)i * 4, sizeof(D[nD].ref));
        ++nD;
    }
    free(pyr);
    if (per_pixel) {
        /* reported per-cell mask: T_H, or a changed pixel of a layer, upsampled, in the cell */
        for (int l = l0; l <= l1; ++l) {
            for (int Y = 0; Y < H; ++Y)
                for (int X = 0; X < W; ++X) {
                    int k = X >> l, m = Y >> l;
                    if (k > lw[l] - 1) k = lw[l] - 1;
                    if (m > lh[l] - 1) m = lh[l] - 1;
                    if (pix[l][m * lw[l] + k]) s->mask[cell_row(Y, H, Nr) * Nc + cell_col(X, W, Nc)] = 1;
                }
            free(pix[l]);
        }
    }
    kp_cmp_ctx_W = W; kp_cmp_ctx_H = H; kp_cmp_ctx_Nc = Nc; kp_cmp_ctx_Nr = Nr; kp_cmp_ctx_layers = s->layers_on;
    qsort(D, (size_t)nD, sizeof(orc_feat), feat_cmp);
    if (nD > s->capK) { free(F); free(D); return -1; }
    for (int i = 0; i < nD; ++i) {
        s->K[i] = D[i].k;
        if (s->desc_on) {
            s->bin[i] = D[i].bin;
            memcpy(s->desc + (size_t)i * 8, D[i].bits, sizeof(D[i].bits));
        }
        if (s->ref_on) memcpy(s->ref + (size_t)i * 4, D[i].ref, sizeof(D[i].ref));
    }
    s->nK = nD;
    for (int c = 0; c < ncell; ++c) s->count[c] = 0;
    for (int i = 0; i < nD; ++i)
        s->count[kp_cell(s->layers_on, &D[i].k, W, H, Nc, Nr)] += 1;
    free(F);
    free(D);

    memcpy(s->prev, frame, (size_t)W * H);
    s->force_all = 0;
    s->n_frames += 1;
    return nD;
}

/* Copy out D_n; mask, per-cell SAD and per-cell counts are optional. */
int orc_get(orc_stream* s, orc_kp* out, int cap, uint8_t* mask, int64_t* sad, uint32_t* count)
{
    int ncell = s->Nc * s->Nr;
    if (out) {
        if (cap < s->nK) return -1;
        memcpy(out, s->K, sizeof(orc_kp) * (size_t)s->nK);
    }
    if (mask) memcpy(mask, s->mask, (size_t)ncell);
    if (sad) memcpy(sad, s->sad, sizeof(int64_t) * (size_t)ncell);
    if (count) memcpy(count, s->count, sizeof(uint32_t) * (size_t)ncell);
    return s->nK;
}

/* ------------------------------------------ temporally coherent detector */

typedef struct {
    int32_t x4, y4, octave, score, sad;
} orc_track;

/* T3 */
static int tcd_sample(const uint8_t* I, int W, int X, int Y)
{
    const int x = X >> 2, y = Y >> 2, a = X & 3, b = Y & 3;
    const int p00 = I[y * W + x];
    const int p10 = a ? I[y * W + x + 1] : 0;
    const int p01 = b ? I[(y + 1) * W + x] : 0;
    const int p11 = (a && b) ? I[(y + 1) * W + x + 1] : 0;
    return ((4 - a) * (4 - b) * p00 + a * (4 - b) * p10 + (4 - a) * b * p01 + a * b * p11 + 8) >> 4;
}

int orc_tcd_sample(const uint8_t* I, int W, int H, int X, int Y)
{
    if (X < 0 || Y < 0 || (X >> 2) + ((X & 3) != 0) >= W || (Y >> 2) + ((Y & 3) != 0) >= H) return -1;
    return tcd_sample(I, W, X, Y);
}

/* T4 */
static int tcd_usable(int W, int H, int X, int Y)
{
    return X >= 32 && Y >= 32 && X + 28 <= 4 * (W - 2) && Y + 28 <= 4 * (H - 2);
}

static void tcd_patch(const uint8_t* I, int W, int X, int Y, int* P)
{
    for (int j = 0; j < 16; ++j)
        for (int i = 0; i < 16; ++i) P[j * 16 + i] = tcd_sample(I, W, X + 4 * (i - 8), Y + 4 * (j - 8));
}

/* T6: the k-th grid offset in spiral order, found by walking the rings */
static void tcd_spiral(int k, int* u, int* v)
{
    int cu = 0, cv = 0, n = 0;
    if (k == 0) { *u = 0; *v = 0; return; }
    n = 1;
    for (int r = 1;; ++r) {
        /* the walk: start at the ring's top-left corner */
        cu = -r; cv = -r;
        static const int du[4] = {1, 0, -1, 0}, dv[4] = {0, 1, 0, -1};
        for (int side = 0; side < 4; ++side)
            for (int step = 0; step < 2 * r; ++step) {
                if (n == k) { *u = cu; *v = cv; return; }
                ++n;
                cu += du[side];
                cv += dv[side];
            }
    }
}

int orc_tcd_spiral(int k, int* u, int* v)
{
    if (k < 0) return -1;
    tcd_spiral(k, u, v);
    return 0;
}

/* one step of T6 around (X, Y): grid of (2R+1)^2 offsets scaled by `scale`
 * quarter pixels; returns the winner's SAD (or -1 with no usable candidate)
 * and its position */
static int tcd_step(const uint8_t* I, int W, int H, const int* ref, int X, int Y, int R, int scale, int t_et,
                    int* bx, int* by)
{
    int best = -1;
    const int n = (2 * R + 1) * (2 * R + 1);
    for (int k = 0; k < n; ++k) {
        int u, v;
        tcd_spiral(k, &u, &v);
        const int cx = X + scale * u, cy = Y + scale * v;
        if (!tcd_usable(W, H, cx, cy)) continue;
        int sad = 0;
        for (int j = 0; j < 16; ++j)
            for (int i = 0; i < 16; ++i) {
                const int d = ref[j * 16 + i] - tcd_sample(I, W, cx + 4 * (i - 8), cy + 4 * (j - 8));
                sad += d < 0 ? -d : d;
            }
        if (best < 0 || sad < best) { best = sad; *bx = cx; *by = cy; }
        if (sad < t_et) break;
    }
    return best;
}

/* T5-T7: propagate n tracks from prev to cur; returns the survivors */
int orc_tcd_track(const uint8_t* prev, const uint8_t* cur, int W, int H, int t_bm, int t_et, const orc_track* in,
                  int n, orc_track* out)
{
    int ref[256], m = 0;
    for (int k = 0; k < n; ++k) {
        const orc_track t = in[k];
        if (!tcd_usable(W, H, t.x4, t.y4)) continue;
        tcd_patch(prev, W, t.x4, t.y4, ref);
        int cx, cy, fx, fy;
        if (tcd_step(cur, W, H, ref, t.x4, t.y4, 6, 8, t_et, &cx, &cy) < 0) continue;
        const int sad = tcd_step(cur, W, H, ref, cx, cy, 7, 1, t_et, &fx, &fy);
        if (sad < 0 || sad >= t_bm) continue;
        out[m] = t;
        out[m].x4 = fx;
        out[m].y4 = fy;
        out[m].sad = sad;
        ++m;
    }
    return m;
}

typedef struct {
    int W, H, gop, t_bm, t_et;
    int n_frames;        /* frames since open or reset */
    orc_stream* det;     /* full-frame detection of the group's first frame (T1) */
    uint8_t* prev;
    orc_track* T;
    orc_track* T2;
    int nT, capT;
} orc_tcd;

orc_tcd* orc_tcd_open(int W, int H, int t, int O, int Nc, int Nr, int gop, int t_bm, int t_et)
{
    if (gop < 1) return NULL;
    orc_stream* det = orc_open(W, H, t, O, Nc, Nr, -1, 0xFFFFFFFFu);
    if (!det) return NULL;
    orc_tcd* s = (orc_tcd*)calloc(1, sizeof(orc_tcd));
    s->W = W; s->H = H; s->gop = gop; s->t_bm = t_bm; s->t_et = t_et;
    s->det = det;
    s->prev = (uint8_t*)malloc((size_t)W * H);
    s->capT = W * H + 16;
    s->T = (orc_track*)malloc(sizeof(orc_track) * (size_t)s->capT);
    s->T2 = (orc_track*)malloc(sizeof(orc_track) * (size_t)s->capT);
    return s;
}

void orc_tcd_close(orc_tcd* s)
{
    if (!s) return;
    orc_close(s->det);
    free(s->prev); free(s->T); free(s->T2);
    free(s);
}

int orc_tcd_reset(orc_tcd* s)
{
    s->n_frames = 0;
    return 0;
}

int orc_tcd_push(orc_tcd* s, const uint8_t* frame)
{
    if (s->n_frames % s->gop == 0) {   /* T1, T2 */
        orc_reset(s->det);
        orc_push(s->det, frame);
        s->nT = 0;
        for (int k = 0; k < s->det->nK; ++k) {
            const orc_kp p = s->det->K[k];
            orc_track* t = &s->T[s->nT++];
            t->x4 = 4 * (p.x << p.octave) + 2 * ((1 << p.octave) - 1);
            t->y4 = 4 * (p.y << p.octave) + 2 * ((1 << p.octave) - 1);
            t->octave = p.octave;
            t->score = p.score;
            t->sad = 0;
        }
    } else {
        const int m = orc_tcd_track(s->prev, frame, s->W, s->H, s->t_bm, s->t_et, s->T, s->nT, s->T2);
        orc_track* x = s->T; s->T = s->T2; s->T2 = x;
        s->nT = m;
    }
    memcpy(s->prev, frame, (size_t)s->W * s->H);
    s->n_frames += 1;
    return s->nT;
}

int orc_tcd_get(orc_tcd* s, orc_track* out, int cap)
{
    if (out) {
        if (cap < s->nT) return -1;
        memcpy(out, s->T, sizeof(orc_track) * (size_t)s->nT);
    }
    return s->nT;
}

/* ------------------------------------------------ intra-octave layers */

/* L1: sizes of the 2O layers in scale order and their pixel sizes in
 * half level-0 pixels; returns the total byte count */
long orc_layer_dims(int W, int H, int O, int* ws, int* hs, int* S)
{
    long total = 0;
    for (int i = 0; i < O; ++i) {
        ws[2 * i] = W >> i;
        hs[2 * i] = H >> i;
        S[2 * i] = 2 << i;
        ws[2 * i + 1] = ((W / 3) * 2) >> i;
        hs[2 * i + 1] = ((H / 3) * 2) >> i;
        S[2 * i + 1] = 3 << i;
        total += (long)ws[2 * i] * hs[2 * i] + (long)ws[2 * i + 1] * hs[2 * i + 1];
    }
    return total;
}

/* L1: the 1.5x downsampling of c_0 into d_0 */
int orc_twothirds(const uint8_t* src, int w, int h, uint8_t* dst)
{
    static const int wt[2][3] = {{2, 1, 0}, {0, 1, 2}};
    const int dw = (w / 3) * 2, dh = (h / 3) * 2;
    for (int Y = 0; Y < dh; ++Y)
        for (int X = 0; X < dw; ++X) {
            const int a = X / 2, p = X % 2, b = Y / 2, q = Y % 2;
            int sum = 0;
            for (int j = 0; j < 3; ++j)
                for (int i = 0; i < 3; ++i) sum += wt[p][i] * wt[q][j] * src[(3 * b + j) * w + 3 * a + i];
            dst[Y * dw + X] = (uint8_t)((sum + 4) / 9);
        }
    return 0;
}

static void halve(const uint8_t* src, int w, int h, uint8_t* dst)
{
    const int dw = w / 2, dh = h / 2;
    for (int y = 0; y < dh; ++y)
        for (int x = 0; x < dw; ++x) {
            const int s = src[2 * y * w + 2 * x] + src[2 * y * w + 2 * x + 1] + src[(2 * y + 1) * w + 2 * x] +
                          src[(2 * y + 1) * w + 2 * x + 1];
            dst[y * dw + x] = (uint8_t)((s + 2) >> 2);
        }
}

/* all 2O layers, concatenated in scale order */
int orc_layers(const uint8_t* img, int W, int H, int O, uint8_t* out)
{
    int ws[64], hs[64], S[64];
    if (O < 1 || O > 16) return -1;
    orc_layer_dims(W, H, O, ws, hs, S);
    long off[65];
    off[0] = 0;
    for (int l = 0; l < 2 * O; ++l) off[l + 1] = off[l] + (long)ws[l] * hs[l];
    memcpy(out, img, (size_t)W * H);
    for (int i = 1; i < O; ++i) halve(out + off[2 * i - 2], ws[2 * i - 2], hs[2 * i - 2], out + off[2 * i]);
    orc_twothirds(img, W, H, out + off[1]);
    for (int i = 1; i < O; ++i) halve(out + off[2 * i - 1], ws[2 * i - 1], hs[2 * i - 1], out + off[2 * i + 1]);
    return 0;
}

static long floor_div(long a, long b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

/* L3: the pixels x' of a layer with pixel size S2 whose footprints meet
 * that of pixel x of pixel size S1: x' S2 <= (x+1) S1 and (x'+1) S2 >= x S1 */
int orc_layer_range(int S1, int S2, int x, int* lo, int* hi)
{
    *lo = (int)(-floor_div(-(long)x * S1, S2)) - 1;   /* ceil(x S1 / S2) - 1 */
    *hi = (int)floor_div((long)(x + 1) * S1, S2);
    return 0;
}

int orc_detect_layers(const uint8_t* img, int W, int H, int t, int O, orc_kp* out, int cap)
{
    int ws[64], hs[64], S[64];
    if (O < 1 || O > 16 || W < 1 || H < 1) return -2;
    const int L = 2 * O;
    long total = orc_layer_dims(W, H, O, ws, hs, S);
    uint8_t* lay = (uint8_t*)malloc((size_t)total + 1);
    uint16_t* V = (uint16_t*)malloc(((size_t)total + 1) * sizeof(uint16_t));
    long off[65];
    off[0] = 0;
    for (int l = 0; l < L; ++l) off[l + 1] = off[l] + (long)ws[l] * hs[l];
    orc_layers(img, W, H, O, lay);
    for (int l = 0; l < L; ++l) orc_score_level(lay + off[l], ws[l], hs[l], t, V + off[l]);
    int n = 0;
    for (int l = 0; l < L; ++l)
        for (int y = 0; y < hs[l]; ++y)
            for (int x = 0; x < ws[l]; ++x) {
                const int v = V[off[l] + (long)y * ws[l] + x];
                if (v == 0) continue;
                int keep = 1;
                for (int m = l - 1; m <= l + 1 && keep; ++m) {
                    if (m < 0 || m >= L) continue;
                    int x0, x1, y0, y1;
                    orc_layer_range(S[l], S[m], x, &x0, &x1);
                    orc_layer_range(S[l], S[m], y, &y0, &y1);
                    for (int qy = y0; qy <= y1 && keep; ++qy)
                        for (int qx = x0; qx <= x1 && keep; ++qx) {
                            if (qx < 0 || qy < 0 || qx >= ws[m] || qy >= hs[m]) continue;
                            if (m == l && qx == x && qy == y) continue;
                            if (beats(V[off[m] + (long)qy * ws[m] + qx], m, qy, qx, v, l, y, x)) keep = 0;
                        }
                }
                if (!keep) continue;
                if (n >= cap) { free(lay); free(V); return -1; }
                out[n].x = x;
                out[n].y = y;
                out[n].octave = l;
                out[n].score = v;
                ++n;
            }
    free(lay);
    free(V);
    return n;
}

/* L4: refined (x, y) in level-0 pixels, log2 scale and score of the
 * keypoint (x, y) of layer l; lay[m], ws[m], hs[m], S[m] describe the
 * 2O layers */
static const double ORC_LOG2_1P5 = 0.58496250072115618;

static double layer_sigma(int m)
{
    /* m = -1 is the intra-octave below c_0, m = L the layer past the last */
    return m % 2 == 0 ? (double)(m / 2) : (double)((m - 1) / 2) + ORC_LOG2_1P5;
}

void orc_refine_layer_kp(uint8_t* const* lay, const int* ws, const int* hs, const int* S, int L, int t, int x, int y,
                         int l, float* out)
{
    double m[3] = {0.0, 0.0, 0.0}, X[3], Y[3], sg[3];
    for (int k = 0; k < 3; ++k) {
        const int ll = l - 1 + k;
        sg[k] = layer_sigma(ll);
        if (ll < 0 || ll >= L) continue;
        const int cx = (int)(((long)(2 * x + 1) * S[l]) / (2L * S[ll]));
        const int cy = (int)(((long)(2 * y + 1) * S[l]) / (2L * S[ll]));
        double u, v;
        fit_patch(lay[ll], ws[ll], hs[ll], t, cx, cy, &u, &v, &m[k]);
        X[k] = (((double)cx + 0.5) + u) * ((double)S[ll] / 2.0);
        Y[k] = (((double)cy + 0.5) + v) * ((double)S[ll] / 2.0);
    }
    if (l == 0) { X[0] = X[1]; Y[0] = Y[1]; }
    if (l + 1 >= L) { X[2] = X[1]; Y[2] = Y[1]; }
    const double d1 = (m[1] - m[0]) / (sg[1] - sg[0]);
    const double d2 = (m[2] - m[1]) / (sg[2] - sg[1]);
    const double a = (d2 - d1) / (sg[2] - sg[0]);
    double sig = sg[1];
    if (a < 0.0) {
        sig = (sg[0] + sg[1]) / 2.0 - d1 / (2.0 * a);
        if (sig > sg[2]) sig = sg[2];
        if (sig < sg[0]) sig = sg[0];
    }
    const double score = (m[0] + d1 * (sig - sg[0])) + (a * (sig - sg[0])) * (sig - sg[1]);
    double px, py;
    if (sig >= sg[1]) {
        const double f = (sig - sg[1]) / (sg[2] - sg[1]);
        px = X[1] + f * (X[2] - X[1]);
        py = Y[1] + f * (Y[2] - Y[1]);
    } else {
        const double f = (sg[1] - sig) / (sg[1] - sg[0]);
        px = X[1] + f * (X[0] - X[1]);
        py = Y[1] + f * (Y[0] - Y[1]);
    }
    out[0] = (float)px;
    out[1] = (float)py;
    out[2] = (float)sig;
    out[3] = (float)score;
}

/* layers of img, then L4 for every keypoint of orc_detect_layers' list */
int orc_refine_layers(const uint8_t* img, int W, int H, int t, int O, const orc_kp* kps, int n, float* out)
{
    int ws[64], hs[64], S[64];
    if (O < 1 || O > 16) return -1;
    const int L = 2 * O;
    long total = orc_layer_dims(W, H, O, ws, hs, S);
    uint8_t* buf = (uint8_t*)malloc((size_t)total + 1);
    orc_layers(img, W, H, O, buf);
    uint8_t* lay[64];
    long off = 0;
    for (int l = 0; l < L; ++l) { lay[l] = buf + off; off += (long)ws[l] * hs[l]; }
    for (int i = 0; i < n; ++i)
        orc_refine_layer_kp(lay, ws, hs, S, L, t, kps[i].x, kps[i].y, kps[i].octave, out + 4 * i);
    free(buf);
    return 0;
}
