// C ABI of the masked multi-scale FAST detector: arena layout, stream state
// and per-frame launch sequence. The declarations and their contracts are in
// include/kpd.h.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <utility>
#include <vector>

#include "../../include/kpd.h"
#include "kpd_errors.h"
#include "kpd_geom.h"
#include "kpd_kernels.h"
#include "kpd_trace.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return KPD_EDEVICE;
}

#define KPD_HIP(call)                                     \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Byte layout of one stream's device arena. Per-frame state that the next
// frame reads is double-buffered: the per-cell SAD by frame parity, the
// per-cell counts and offsets and the keypoint list D_n by alternation (the
// stream remembers which buffer holds the latest D_n).
struct Layout {
    int W = 0, H = 0, O = 0, nc = 0, nr = 0, ncell = 0;
    int w[KPD_MAX_OCTAVES] = {}, h[KPD_MAX_OCTAVES] = {}, pitch[KPD_MAX_OCTAVES] = {};
    int slot_pitch = 0;
    int tile = 32;       // level-0 tile side of the pyramid/SAD workgroups
    int tiles_x = 0, tiles_y = 0;
    int sad_slots = 1;   // cells one tile can touch
    size_t off_hdr = 0, off_slot[2] = {0, 0}, off_lvl[KPD_MAX_OCTAVES] = {};
    size_t off_sad[2] = {0, 0}, off_count[2] = {0, 0}, off_offs[2] = {0, 0}, off_list[2] = {0, 0};
    size_t off_mask = 0, off_status = 0, off_colw = 0, off_rowh = 0, off_layouts = 0;
    size_t off_colmap = 0, off_rowmap = 0;   // cell column / row of every level-0 column / row
    // batch ticks: marked cells' keypoints at fixed per-cell bases, and counts
    size_t off_sparse1 = 0, off_own1 = 0;
    size_t off_desc[2] = {0, 0}, off_dtab = 0;   // descriptors (KPD_FEAT_DESCRIPTOR)
    size_t off_ref[2] = {0, 0};                  // refined values (KPD_FEAT_REFINE)
    // chunks of consecutive frames (push_frames): K copies of the octaves,
    // per-frame SAD, sparse lists with per-cell counts, count words, marks
    // (cell-major, Kw 64-bit words per cell), dense lists with counts, offsets and
    // totals, the cells' sparse bases, and the fixed per-frame argument
    // tables of the tile and detection passes
    int K = 1, Kw = 1;
    int ctile = 32, ctiles_x = 0, ctiles_y = 0, csad_slots = 1;   // tile pass of chunks
    bool seq_ok = false;   // the sequential tile pass of chunks can run (k_frame_chunk_seq)
    int seq_tile_w = 256, seq_tiles_x = 0, seq_ntiles = 0, seq_slots = 1;   // its tiles, LDS slots a tile
    size_t pyr_stride = 0;
    size_t off_csad = 0, off_ccount = 0, off_coffs = 0, off_ctotal = 0, off_clist = 0, clist_stride = 0;
    size_t off_cdesc = 0, off_cref = 0;   // features of chunk frames 0..K-2 (clist_stride entries apart)
    size_t off_sparse = 0, off_own = 0, off_marks = 0, off_cbase = 0, off_work = 0;
    size_t off_ctab = 0;
    size_t list_cap = 0;    // entries of chunk and sparse lists: one feature per 2x2 decision block
    size_t list_cap1 = 0;   // entries of the single-frame D lists: every decision pixel with layer_mask
    int lds_bytes = 0;   // dynamic LDS of the cell pass
    // the per-pixel layer mask (set_mask_mode): its LDS scratch past every
    // cell's layout (changed bits, carried bits, their offsets and scores),
    // and a second buffer for octave 1.. so the layer of I_{n-1} survives
    int lds_bits = 0, lds_carr = 0, lds_cwoff = 0, lds_cscore = 0, lds_csrc = 0, lds_bytes1 = 0;
    size_t off_src = 0;   // features with a per-pixel mask: each D_n entry's source
    size_t off_lvl_alt = 0;
    // per-pixel masks in chunks (layer_mask streams): the cells' layer-pixel
    // change bits (fpw words per frame and cell) and change flags, the
    // merged lists (decision-pixel bases pbase), their counts, and the
    // merge pass's LDS
    int fpw = 0, nwords_max = 0, dc_max = 0;
    size_t off_pflag = 0, off_fp = 0, off_msparse = 0, off_mcount = 0, off_pbase = 0;
    int pm_pres = 0, pm_score = 0, pm_fp = 0, pm_ents = 0, pm_lds = 0, pm_batch = 1;
    int pm_tgate = 0, pm_txy = 0, pm_toct = 0, pm_tab = 0, pm_tsrc = 0;
    size_t off_msrc = 0, off_sdesc = 0, off_sref = 0;   // features with a per-pixel mask in chunks
    // the group detector of full-frame chunks: gx x gy cells per workgroup
    // and the groups' layouts
    int gx = 1, gy = 1, ngroups = 0, glds = 0, gthreads = 256;
    size_t off_glay = 0;
    // single frames: one-cell layouts of the same detector, and its LDS at
    // 256 and 512 threads
    size_t off_glay1 = 0;
    int glds1_128 = 0, glds1_256 = 0, glds1_512 = 0;
    int glds1_1024 = 0;   // 0: one cell does not fit a 1024-thread workgroup's LDS
    size_t total = 0;
};

// header words
constexpr int kHdrTotal0 = 0, kHdrTotal1 = 1, kHdrErr = 3, kHdrWork = 4;   // kHdrWork + 1: a chunk's second work count
constexpr size_t kStage = 4096;   // D_n entries staged by get_keypoints

bool valid_params(int W, int H, const kpd_params* p, std::string* why)
{
    if (!p) { *why = "params is NULL"; return false; }
    if (W < 1 || H < 1 || W > KPD_MAX_DIM || H > KPD_MAX_DIM) { *why = "frame size out of range"; return false; }
    if (p->fast_t < 1 || p->fast_t > 254) { *why = "fast_t must be in 1..254"; return false; }
    if (p->n_octaves < 1 || p->n_octaves > KPD_MAX_OCTAVES) { *why = "n_octaves out of range"; return false; }
    if ((W >> (p->n_octaves - 1)) < 1 || (H >> (p->n_octaves - 1)) < 1) {
        *why = "frame too small for n_octaves";
        return false;
    }
    if (p->grid_cols < 1 || p->grid_rows < 1 || p->grid_cols > W || p->grid_rows > H) {
        *why = "grid out of range";
        return false;
    }
    if (kpd::ceil_div(W, p->grid_cols) > KPD_MAX_CELL || kpd::ceil_div(H, p->grid_rows) > KPD_MAX_CELL) {
        *why = "cells larger than KPD_MAX_CELL pixels";
        return false;
    }
    if (p->tile != 0 && (p->tile < 32 || p->tile > 128 || (p->tile & (p->tile - 1)) ||
                         p->tile < (1 << (p->n_octaves - 1)))) {
        *why = "tile must be 0 or a power of two in 32..128 and >= 2^(O-1)";
        return false;
    }
    if (p->chunk_frames < 0 || p->chunk_frames > KPD_MAX_CHUNK) {
        *why = "chunk_frames out of range";
        return false;
    }
    if (p->layer_mask != 0 && p->layer_mask != 1) { *why = "layer_mask must be 0 or 1"; return false; }
    if (p->features & ~(KPD_FEAT_DESCRIPTOR | KPD_FEAT_REFINE)) { *why = "unknown feature bits"; return false; }
    if ((p->group_cols == 0) != (p->group_rows == 0) || p->group_cols < 0 || p->group_rows < 0 ||
        p->group_cols > p->grid_cols || p->group_rows > p->grid_rows) {
        *why = "group_cols and group_rows must both be 0 or in 1..grid_cols and 1..grid_rows";
        return false;
    }
    if (p->group_cols * p->group_rows > kpd::kGroupMaxCells) {
        *why = "at most " + std::to_string(kpd::kGroupMaxCells) + " cells per group";
        return false;
    }
    if (p->group_threads != 0 && p->group_threads != 256 && p->group_threads != 512) {
        *why = "group_threads must be 0, 256 or 512";
        return false;
    }
    return true;
}

// Layouts of every group of gx x gy cells (row-major over the group grid);
// false when a group is too large for the detector. *lds: the largest
// workgroup LDS need at `waves` waves.
// Each cell's first entry in a keypoint list of one feature per 2x2 block
// of its decision boxes (cells in row-major order).
std::vector<uint32_t> cell_bases(const Layout& L)
{
    std::vector<uint32_t> base(L.ncell);
    uint32_t acc = 0;
    for (int c = 0; c < L.ncell; ++c) {
        base[c] = acc;
        const kpd::Box r = kpd::cell_rect(c, L.W, L.H, L.nc, L.nr);
        for (int o = 0; o < L.O; ++o) acc += (uint32_t)kpd::decision_capacity(kpd::decision_box(r, o, L.w[o], L.h[o]));
    }
    return base;
}

bool group_layouts(const Layout& L, int gx, int gy, int waves, std::vector<kpd::GroupLayout>* out, int* lds)
{
    const int ngc = (L.nc + gx - 1) / gx, ngr = (L.nr + gy - 1) / gy;
    if (out) out->assign((size_t)ngc * ngr, kpd::GroupLayout{});
    const std::vector<uint32_t> bases = out ? cell_bases(L) : std::vector<uint32_t>();
    *lds = 0;
    for (int r = 0; r < ngr; ++r)
        for (int q = 0; q < ngc; ++q) {
            const int c0 = q * gx, c1 = std::min(c0 + gx, L.nc), r0 = r * gy, r1 = std::min(r0 + gy, L.nr);
            const kpd::Box a = kpd::cell_rect(r0 * L.nc + c0, L.W, L.H, L.nc, L.nr);
            const kpd::Box b = kpd::cell_rect((r1 - 1) * L.nc + c1 - 1, L.W, L.H, L.nc, L.nr);
            kpd::GroupLayout G;
            if (!kpd::group_layout(kpd::Box{a.x0, b.x1, a.y0, b.y1}, L.O, L.w, L.h, c0, c1, r0, r1, L.W, L.H, L.nc,
                                   L.nr, out ? bases.data() : nullptr, &G))
                return false;
            *lds = std::max(*lds, kpd::group_lds_bytes(G, waves));
            if (out) (*out)[(size_t)r * ngc + q] = G;
        }
    return true;
}

constexpr int kGroupWaves = 4;           // 256-thread workgroups for one-cell layouts
constexpr int kGroupLdsDefault = 48 * 1024;   // default groups: three workgroups per CU
constexpr uint32_t kPixelStagedMaxima = 1024;  // maxima of a batch the per-pixel merge stages in LDS

// Threads of a workgroup of the listed-cell detection of chunks. Few cells
// a frame mean few listed items, whose latency decides: more waves per item
// shorten its chain; many cells mean many items, whose throughput decides:
// smaller workgroups keep more of them in flight. Measured on the masked
// videos (listed detection per 300 frames): 640x480 with 192 cells 17.3,
// 18.9 and 24.4 us at 512, 256 and 128 threads (26.3 at 1024, one
// workgroup per CU); 1920x1080 with 576 cells 245, 172 and 162 us.
int list_threads(const Layout& L)
{
    return L.ncell <= 256 ? 512 : (L.ncell >= 512 ? 128 : 256);
}

// Dynamic LDS of a one-cell group workgroup of `threads` threads (its wave
// queues scale with the waves).
int glds1_for(const Layout& L, int threads)
{
    return threads == 128 ? L.glds1_128
                          : (threads == 512 ? L.glds1_512 : (threads == 1024 ? L.glds1_1024 : L.glds1_256));
}

// Whether the sequential tile pass takes this geometry: octaves to level 5
// (O <= 6), the frame width a multiple of 16, every 16-column segment in at
// most two cell columns, each dword in one, and every block of 4 rows (its
// rows inside the frame) in at most two cell rows: the kernel sums such a
// block in four registers. Column X is in cell column floor(X Nc / W), row
// Y in cell row floor(Y Nr / H).
bool seq_geometry_ok(const Layout& L)
{
    if (L.O > 6 || L.W % 16 != 0) return false;
    auto ccol = [&](int x) { return (int)(((int64_t)x * L.nc) / L.W); };
    auto crow = [&](int y) { return (int)(((int64_t)y * L.nr) / L.H); };
    for (int x = 0; x < L.W; x += 16) {
        for (int d = 0; d < 4; ++d)
            if (ccol(x + 4 * d) != ccol(x + 4 * d + 3)) return false;
        if (ccol(x + 15) - ccol(x) > 1) return false;
    }
    for (int y = 0; y < L.H; y += 4)
        if (crow(std::min(y + 3, L.H - 1)) - crow(y) > 1) return false;
    return true;
}

bool make_layout(int W, int H, const kpd_params* p, Layout* L, std::string* why)
{
    if (!valid_params(W, H, p, why)) return false;
    L->W = W; L->H = H; L->O = p->n_octaves; L->nc = p->grid_cols; L->nr = p->grid_rows;
    L->ncell = L->nc * L->nr;
    for (int o = 0; o < L->O; ++o) {
        L->w[o] = W >> o;
        L->h[o] = H >> o;
        // whole 128-byte lines per level row: the tile passes write each
        // row in aligned runs, which neighbouring tiles complete in the L2
        L->pitch[o] = kpd::round_up(L->w[o], 128);
    }
    L->slot_pitch = kpd::round_up(W, 64);
    // cells a k_frame tile can touch, per axis
    auto span_max = [](int len, int n, int T) {
        int m = 1;
        for (int x0 = 0; x0 < len; x0 += T) {
            const int x1 = std::min(x0 + T, len) - 1;
            m = std::max(m, (int)(((int64_t)x1 * n) / len) - (int)(((int64_t)x0 * n) / len) + 1);
        }
        return m;
    };
    // Single frames: the widest tile that still gives at least 128
    // workgroups (a frame's tile pass is short; wider tiles cost fewer
    // workgroups per byte), at least 32 and 2^(O-1) pixels a side.
    L->tile = p->tile;
    if (!L->tile) {
        const int tmin = std::max(32, 1 << (L->O - 1));
        L->tile = tmin;
        for (int T = 128; T > tmin; T >>= 1) {
            const int nt = ((W + T - 1) / T) * ((H + T - 1) / T);
            const int slots = span_max(W, L->nc, T) * span_max(H, L->nr, T);
            if (nt >= 128 && kpd::frame_lds_bytes(T, L->O, slots) <= 65536) {
                L->tile = T;
                break;
            }
        }
    }
    L->tiles_x = (W + L->tile - 1) / L->tile;
    L->tiles_y = (H + L->tile - 1) / L->tile;
    L->sad_slots = span_max(W, L->nc, L->tile) * span_max(H, L->nr, L->tile);
    if (kpd::frame_lds_bytes(L->tile, L->O, L->sad_slots) > 65536) {
        *why = "grid too fine for the pyramid tile";
        return false;
    }
    // A chunk has many frames' tiles to spread over the chip, so its tile
    // pass takes the widest tile that fits (whole 128-byte rows per tile
    // row); a single frame keeps the smaller tile for more workgroups.
    L->ctile = L->tile;
    for (int T = 128; T > L->tile; T >>= 1) {
        const int slots = span_max(W, L->nc, T) * span_max(H, L->nr, T);
        if (kpd::frame_lds_bytes(T, L->O, slots) <= 65536) {
            L->ctile = T;
            break;
        }
    }
    L->ctiles_x = (W + L->ctile - 1) / L->ctile;
    L->ctiles_y = (H + L->ctile - 1) / L->ctile;
    L->csad_slots = span_max(W, L->nc, L->ctile) * span_max(H, L->nr, L->ctile);
    L->seq_ok = seq_geometry_ok(*L);
    // 256 x 64 tiles (level-1 rows in whole lines) when their octaves reach
    // far enough and at most a tenth of the last tile column lies past the
    // frame, else 128 x 128
    const int pad256 = (W + 255) / 256 * 256 - W;
    L->seq_tile_w = (L->O <= 5 && pad256 * 10 <= W) ? 256 : 128;
    const int seq_th = 4 * (256 / (L->seq_tile_w / 16));
    L->seq_tiles_x = (W + L->seq_tile_w - 1) / L->seq_tile_w;
    L->seq_ntiles = L->seq_tiles_x * ((H + seq_th - 1) / seq_th);
    L->seq_slots = span_max(W, L->nc, L->seq_tile_w) * span_max(H, L->nr, seq_th);

    // keypoint list capacity and the detection kernel's LDS need
    size_t cap = 0, dec_px = 0;
    int lds = 0, nwords_max = 0, npx_max = 0;
    size_t cell_cap_max = 0;
    for (int c = 0; c < L->ncell; ++c) {
        const kpd::Box r = kpd::cell_rect(c, W, H, L->nc, L->nr);
        kpd::CellLayout CL;
        kpd::cell_layout(r, L->O, L->w, L->h, &CL);
        size_t cc = 0;
        for (int o = 0; o < L->O; ++o) cc += kpd::decision_capacity(CL.dec[o]);
        cap += cc;
        dec_px += (size_t)CL.dc_start[L->O];
        cell_cap_max = std::max(cell_cap_max, p->layer_mask ? (size_t)CL.dc_start[L->O] : cc);
        nwords_max = std::max(nwords_max, CL.nwords);
        int npx_sum = 0;   // layer pixels the cell maps to, summed over the layers, each rounded up to 64
        for (int lv = 0; lv < L->O; ++lv) {
            const int nx = std::min((r.x1 - 1) >> lv, L->w[lv] - 1) - std::min(r.x0 >> lv, L->w[lv] - 1) + 1;
            const int ny = std::min((r.y1 - 1) >> lv, L->h[lv] - 1) - std::min(r.y0 >> lv, L->h[lv] - 1) + 1;
            npx_sum += kpd::round_up(nx * ny, 64);
        }
        npx_max = std::max(npx_max, npx_sum);
        lds = std::max(lds, CL.bytes);
        // the detection kernel queues score-pixel indices as 16-bit values
        if (CL.sc_start[L->O] > 65535) { *why = "cell too large"; return false; }
        if (cap > 0xFFFFFFF0ull) { *why = "keypoint list too large"; return false; }
    }
    L->list_cap = std::max<size_t>(cap, 1);
    L->list_cap1 = p->layer_mask ? std::max<size_t>(dec_px, 1) : L->list_cap;
    L->fpw = npx_max / 64;
    L->nwords_max = nwords_max;
    L->dc_max = (int)cell_cap_max;
    L->pm_pres = 0;
    L->pm_score = kpd::round_up(nwords_max * 8, 16);
    L->pm_fp = kpd::round_up(L->pm_score + (int)cell_cap_max * 2, 16);
    // the decision-pixel tables (7 bytes a pixel) when they leave room for
    // one frame's change words; then frames whose change words the merge
    // stages at once: about 24 KB, less when the rest leaves less of the
    // 60 KB the pass may take
    const int dcm = (int)cell_cap_max;
    const int tab_bytes = kpd::round_up(dcm * 2, 16) + kpd::round_up(dcm * 4, 16) + kpd::round_up(dcm, 16);
    const int ents_bytes = kpd::round_up((int)kPixelStagedMaxima * (int)sizeof(kpd_keypoint), 16);
    const int src_bytes = p->features ? kpd::round_up(dcm * 4, 16) : 0;   // each map entry's source
    const int fixed = L->pm_fp + ents_bytes + src_bytes + 16;
    L->pm_tab = (fixed + kpd::round_up(L->fpw * 8, 16) + tab_bytes <= 60 * 1024 && L->fpw * 64 <= 65536) ? 1 : 0;
    const int pm_room = 60 * 1024 - fixed - (L->pm_tab ? tab_bytes : 0);
    L->pm_batch = std::max(1, std::min(32, std::min(24 * 1024, pm_room) / std::max(1, L->fpw * 8)));
    L->pm_ents = kpd::round_up(L->pm_fp + L->pm_batch * L->fpw * 8, 16);
    L->pm_tgate = L->pm_ents + ents_bytes;
    L->pm_txy = L->pm_tgate + kpd::round_up(dcm * 2, 16);
    L->pm_toct = L->pm_txy + kpd::round_up(dcm * 4, 16);
    L->pm_tsrc = L->pm_tab ? L->pm_toct + kpd::round_up(dcm, 16) : L->pm_tgate;
    L->pm_lds = L->pm_tsrc + src_bytes;
    if (L->list_cap1 > 0xFFFFFFF0ull) { *why = "keypoint list too large"; return false; }
    L->lds_bytes = std::max(lds, 16);
    {
        int o1 = kpd::round_up(lds, 16);
        L->lds_bits = o1;   o1 += kpd::round_up(npx_max / 8, 16);
        L->lds_carr = o1;   o1 += kpd::round_up(nwords_max * 8, 16);
        L->lds_cwoff = o1;  o1 += kpd::round_up(nwords_max * 4, 16);
        L->lds_cscore = o1; o1 += kpd::round_up((int)cell_cap_max * 2, 16);
        L->lds_csrc = o1;
        if (p->features) o1 += kpd::round_up((int)cell_cap_max * 4, 16);   // carried entries' sources
        L->lds_bytes1 = o1;
    }

    L->K = std::max(1, (int)p->chunk_frames);

    // groups of the full-frame chunk detector: the given shape, or the widest
    // run of cells along a cell row (a power of two) that fits the default LDS
    if (L->K > 1) {
        int lds = 0;
        L->gthreads = p->group_threads ? p->group_threads : 256;
        const int waves = L->gthreads / 64;
        if (p->group_cols > 0) {
            L->gx = p->group_cols;
            L->gy = p->group_rows;
            if (!group_layouts(*L, L->gx, L->gy, waves, nullptr, &lds) || lds > 160 * 1024) {
                *why = "group of cells too large for one workgroup";
                return false;
            }
        } else {
            L->gx = L->gy = 1;
            if (!group_layouts(*L, 1, 1, waves, nullptr, &lds) || lds > 160 * 1024) {
                *why = "cells too large for the group detector";
                return false;
            }
            for (int g = 2; g <= L->nc && g <= kpd::kGroupMaxCells; g *= 2) {
                int l2 = 0;
                if (!group_layouts(*L, g, 1, waves, nullptr, &l2) || l2 > kGroupLdsDefault) break;
                L->gx = g;
                lds = l2;
            }
        }
        L->glds = lds;
        L->ngroups = ((L->nc + L->gx - 1) / L->gx) * ((L->nr + L->gy - 1) / L->gy);
    }
    if (!group_layouts(*L, 1, 1, 2, nullptr, &L->glds1_128) || !group_layouts(*L, 1, 1, 4, nullptr, &L->glds1_256) ||
        !group_layouts(*L, 1, 1, 8, nullptr, &L->glds1_512) ||
        L->glds1_512 > 160 * 1024) {
        *why = "cells too large for the detector";
        return false;
    }
    if (!group_layouts(*L, 1, 1, 16, nullptr, &L->glds1_1024) || L->glds1_1024 > 160 * 1024) L->glds1_1024 = 0;

    size_t off = 0;
    L->off_hdr = off; off = align_up(off + 64);
    for (int k = 0; k < 2; ++k) { L->off_slot[k] = off; off = align_up(off + (size_t)L->slot_pitch * H); }
    const size_t pyr0 = off;
    for (int o = 1; o < L->O; ++o) { L->off_lvl[o] = off; off = align_up(off + (size_t)L->pitch[o] * L->h[o]); }
    L->pyr_stride = off - pyr0;
    off += L->pyr_stride * (size_t)(L->K - 1);   // octave copies of chunk frames 1..K-1
    // a second copy of octaves 1..O-1 for the per-pixel masks, which read the
    // previous frame's levels while the current frame's are written
    if (L->O > 1 && p->layer_mask) { L->off_lvl_alt = off; off = align_up(off + L->pyr_stride); }
    const size_t nc4 = (size_t)L->ncell * 4;
    for (int k = 0; k < 2; ++k) { L->off_sad[k] = off; off = align_up(off + nc4); }
    for (int k = 0; k < 2; ++k) { L->off_count[k] = off; off = align_up(off + nc4); }
    for (int k = 0; k < 2; ++k) { L->off_offs[k] = off; off = align_up(off + nc4); }
    L->off_mask = off; off = align_up(off + (size_t)L->ncell);
    L->off_status = off; off = align_up(off + (size_t)L->ncell * 8);
    L->off_colw = off; off = align_up(off + (size_t)L->nc * 2);
    L->off_rowh = off; off = align_up(off + (size_t)L->nr * 2);
    L->off_colmap = off; off = align_up(off + (size_t)W * 2);
    L->off_rowmap = off; off = align_up(off + (size_t)H * 2);
    L->off_layouts = off; off = align_up(off + (size_t)L->ncell * sizeof(kpd::CellLayout));
    for (int k = 0; k < 2; ++k) {
        L->off_list[k] = off;
        off = align_up(off + L->list_cap1 * sizeof(kpd_keypoint));
    }
    L->off_cbase = off; off = align_up(off + (size_t)L->ncell * 4);
    L->off_own1 = off; off = align_up(off + (size_t)L->ncell * 4);
    L->off_sparse1 = off; off = align_up(off + L->list_cap1 * sizeof(kpd_keypoint));
    L->off_glay1 = off; off = align_up(off + (size_t)L->ncell * sizeof(kpd::GroupLayout));
    if (p->features & KPD_FEAT_DESCRIPTOR) {   // descriptors of D_{n-1} and D_n, and the pattern tables
        for (int k = 0; k < 2; ++k) { L->off_desc[k] = off; off = align_up(off + L->list_cap1 * sizeof(kpd_descriptor)); }
        L->off_dtab = off; off = align_up(off + sizeof(kpd::DescTables));
    }
    if (p->features && p->layer_mask) { L->off_src = off; off = align_up(off + L->list_cap1 * 4); }
    if (p->features & KPD_FEAT_REFINE)   // refined values of D_{n-1} and D_n
        for (int k = 0; k < 2; ++k) { L->off_ref[k] = off; off = align_up(off + L->list_cap1 * sizeof(kpd_refined)); }
    if (L->K > 1) {
        const size_t kc = (size_t)L->K * L->ncell;
        L->off_csad = off; off = align_up(off + kc * 4);
        L->off_ccount = off; off = align_up(off + kc * 4);
        L->off_coffs = off; off = align_up(off + kc * 4);
        L->off_ctotal = off; off = align_up(off + (size_t)L->K * 4);
        L->Kw = (L->K + 63) / 64;
        L->off_marks = off; off = align_up(off + (size_t)L->ncell * L->Kw * 8);
        L->off_own = off; off = align_up(off + kc * 4);
        L->off_work = off; off = align_up(off + kc * 4);
        // with the per-pixel mask a frame's list may hold an entry per decision pixel
        L->clist_stride = align_up((p->layer_mask ? L->list_cap1 : L->list_cap) * sizeof(kpd_keypoint));
        L->off_sparse = off; off += L->clist_stride * (size_t)L->K;
        L->off_clist = off; off += L->clist_stride * (size_t)(L->K - 1);   // the last frame's D goes to D_n
        const size_t centries = L->clist_stride / sizeof(kpd_keypoint) * (size_t)(L->K - 1);
        if (p->features & KPD_FEAT_DESCRIPTOR) { L->off_cdesc = off; off = align_up(off + centries * sizeof(kpd_descriptor)); }
        if (p->features & KPD_FEAT_REFINE) { L->off_cref = off; off = align_up(off + centries * sizeof(kpd_refined)); }
        if (p->layer_mask && p->features) {
            L->off_msrc = off; off = align_up(off + (L->clist_stride / sizeof(kpd_keypoint)) * (size_t)L->K * 4);
            if (p->features & KPD_FEAT_DESCRIPTOR) {
                L->off_sdesc = off; off = align_up(off + L->list_cap * (size_t)L->K * sizeof(kpd_descriptor));
            }
            if (p->features & KPD_FEAT_REFINE) {
                L->off_sref = off; off = align_up(off + L->list_cap * (size_t)L->K * sizeof(kpd_refined));
            }
        }
        if (p->layer_mask) {
            L->off_pflag = off; off = align_up(off + kc * 4);
            L->off_fp = off; off = align_up(off + kc * (size_t)L->fpw * 8);
            L->off_msparse = off; off += L->clist_stride * (size_t)L->K;
            L->off_mcount = off; off = align_up(off + kc * 4);
            L->off_pbase = off; off = align_up(off + (size_t)L->ncell * 4);
        }
        L->off_ctab = off; off = align_up(off + (size_t)L->K * sizeof(kpd::ChunkArgs));
        L->off_glay = off; off = align_up(off + (size_t)L->ngroups * sizeof(kpd::GroupLayout));
    }
    L->total = off;
    return true;
}

// Opt-in per-kernel timing with event pairs recorded around each launch.
struct KernelTimer {
    bool on = false;
    std::vector<hipEvent_t> free_events;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    double ms[KPD_NKERNELS] = {};
    uint64_t launches[KPD_NKERNELS] = {};

    hipError_t take(hipEvent_t* e)
    {
        if (!free_events.empty()) {
            *e = free_events.back();
            free_events.pop_back();
            return hipSuccess;
        }
        return hipEventCreate(e);
    }
    ~KernelTimer()
    {
        // teardown: nothing to report a failure to
        for (auto& p : pending) { (void)hipEventDestroy(p.second.first); (void)hipEventDestroy(p.second.second); }
        for (auto e : free_events) (void)hipEventDestroy(e);
    }
};

}  // namespace

struct kpd_stream {
    Layout L;
    KernelTimer timer;
    kpd_params p{};
    hipStream_t stream = nullptr;
    uint8_t* arena = nullptr;
    int n_pushed = 0;
    bool force_all = true;
    int cur_slot = 0;
    const uint8_t* prev0 = nullptr;
    int prev_pitch = 0;
    int prev_dw = 0;
    int fb_last = 1;          // which of the two single-frame buffers holds the latest D_n
    int det1_threads = 512;   // workgroup size of a single frame's marked cells
    int seq_cap = 0;          // resident workgroups of the sequential chunk tile pass (0: not asked yet)
    int id_mode = 0;          // 0: per-cell mean difference at level 0; 1: per-pixel on layer id_layer;
                              // 2: per-pixel on every level, one mask per octave
    int id_layer = 0;
    int layer_buf = 0;        // the mask's octaves >= 1 of the latest frame: 0 their usual buffers, 1 the second copy
    int chunk_n = 0;          // frames of the last push_frames call
    std::vector<kpd::GroupLayout> glay;   // the group detector's layouts (chunks)
    std::vector<kpd::GroupLayout> glay1;  // its one-cell layouts (single frames)
    kpd::FrameArgs chunk_fa{};  // tile-pass arguments of chunk frame 0
    kpd_batch* batch = nullptr;   // the batch it is attached to
    // pinned host staging for get_keypoints: header, the first kStage
    // entries of D_n and the mask come back in one round trip
    uint8_t* stage = nullptr;       // pinned host staging of get_keypoints
    uint8_t* stage_dev = nullptr;   // its address on the device

    ~kpd_stream()
    {
        if (stage) (void)hipHostFree(stage);
    }

    template <typename T>
    T* at(size_t off) const { return reinterpret_cast<T*>(arena + off); }
};

namespace {

// Launch one kernel of the frame, bracketed by events when timing is on.
template <typename F>
hipError_t timed(kpd_stream* s, int kernel, F&& launch)
{
    if (!s->timer.on) return launch();
    hipEvent_t a, b;
    hipError_t e = s->timer.take(&a);
    if (e == hipSuccess) e = s->timer.take(&b);
    if (e != hipSuccess) return e;
    e = hipEventRecord(a, s->stream);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, s->stream);
    s->timer.pending.push_back({kernel, {a, b}});
    return e;
}

// A level-0 frame can be read a dword at a time when its base and pitch are
// 4-byte aligned and no dword of a row reaches past the row's last byte
// (width a multiple of 4), or when it is one of the arena's padded slots.
int dword_readable(const void* p, int pitch, int width, bool slot)
{
    if (slot) return 1;
    return (reinterpret_cast<uintptr_t>(p) % 4 == 0 && pitch % 4 == 0 && width % 4 == 0) ? 1 : 0;
}

}  // namespace

extern "C" {

const char* kpd_last_error(void) { return g_err.c_str(); }

size_t stream_bytes(int width, int height, const kpd_params* params)
{
    Layout L;
    std::string why;
    if (!make_layout(width, height, params, &L, &why)) {
        g_err = why;
        return 0;
    }
    return L.total;
}

}  // extern "C"

namespace {

// The descriptor pattern (the feature model of Sec. 3; kpd.h states the
// pattern): 60 points, the centre and four rings, turned to each of 32
// sectors and rounded half away from zero; the long pairs (squared distance
// >= 169 between the unturned points) with their offset difference; the 512
// shortest pairs (squared distance < 96, by distance, then indices); the
// sector boundary vectors round(2^20 (cos, sin)).
void build_desc_tables(kpd::DescTables* T)
{
    static const double kR[5] = {0.0, 3.0, 5.0, 7.5, 11.0};
    static const int kN[5] = {1, 10, 14, 15, 20}, kH[5] = {1, 1, 1, 2, 2};
    std::memset(T, 0, sizeof(*T));
    for (int b = 0; b < kpd::kDescSectors; ++b) {
        int i = 0;
        for (int r = 0; r < 5; ++r)
            for (int k = 0; k < kN[r]; ++k, ++i) {
                const double a = (2.0 * M_PI * k) / kN[r] + (2.0 * M_PI * b) / kpd::kDescSectors;
                T->pt[b][i][0] = (int8_t)std::lround(kR[r] * std::cos(a));
                T->pt[b][i][1] = (int8_t)std::lround(kR[r] * std::sin(a));
                T->half[i] = (uint8_t)kH[r];
            }
        T->ux[b] = std::llround(1048576.0 * std::cos((2.0 * M_PI * b) / kpd::kDescSectors));
        T->uy[b] = std::llround(1048576.0 * std::sin((2.0 * M_PI * b) / kpd::kDescSectors));
    }
    struct Pair { int d2, a, b; };
    std::vector<Pair> shorts;
    for (int a = 0; a < kpd::kDescPts; ++a)
        for (int b = a + 1; b < kpd::kDescPts; ++b) {
            const int dx = T->pt[0][b][0] - T->pt[0][a][0], dy = T->pt[0][b][1] - T->pt[0][a][1];
            const int d2 = dx * dx + dy * dy;
            if (d2 >= 169) {
                T->lp[T->nlong][0] = (uint8_t)a;
                T->lp[T->nlong][1] = (uint8_t)b;
                T->ld[T->nlong][0] = (int8_t)dx;
                T->ld[T->nlong][1] = (int8_t)dy;
                ++T->nlong;
            }
            if (d2 < 96) shorts.push_back({d2, a, b});
        }
    std::sort(shorts.begin(), shorts.end(), [](const Pair& x, const Pair& y) {
        return x.d2 != y.d2 ? x.d2 < y.d2 : (x.a != y.a ? x.a < y.a : x.b < y.b);
    });
    for (int k = 0; k < kpd::kDescBits; ++k) {
        T->sp[k][0] = (uint8_t)shorts[k].a;
        T->sp[k][1] = (uint8_t)shorts[k].b;
    }
}

const kpd::DescTables& desc_tables()
{
    static const kpd::DescTables* t = [] {
        auto* p = new kpd::DescTables;
        build_desc_tables(p);
        return p;
    }();
    return *t;
}

// Fixed per-frame arguments of the chunk passes: frame j's octave copy, SAD
// accumulators, sparse list, count words and marks. What changes between
// chunks travels in the ChunkHead kernel argument. The tile pass takes
// frame 0's FrameArgs and steps to frame j's octaves and SAD itself.
void chunk_tables(kpd_stream* s, std::vector<kpd::ChunkArgs>* ctab, std::vector<kpd::FrameArgs>* ftab)
{
    const Layout& L = s->L;
    const size_t kc = (size_t)L.ncell;
    ctab->assign(L.K, kpd::ChunkArgs{});
    ftab->assign(L.K, kpd::FrameArgs{});
    for (int j = 0; j < L.K; ++j) {
        uint8_t* pyr = s->arena + L.pyr_stride * (size_t)j;
        kpd::FrameArgs& fa = (*ftab)[j];
        for (int o = 1; o < L.O; ++o) {
            fa.lvl[o] = pyr + L.off_lvl[o];
            fa.pitch[o] = L.pitch[o];
        }
        for (int o = 0; o < L.O; ++o) { fa.w[o] = L.w[o]; fa.h[o] = L.h[o]; }
        fa.W = L.W; fa.H = L.H; fa.O = L.O; fa.nc = L.nc; fa.nr = L.nr;
        fa.tile = L.ctile;
        fa.tiles_x = L.ctiles_x;
        fa.ntiles = L.ctiles_x * L.ctiles_y;
        fa.sad_slots = L.csad_slots;
        fa.sad_lds_off = kpd::frame_sad_lds_off(L.ctile, L.O);
        fa.sad = s->at<uint32_t>(L.off_csad) + (size_t)j * kc;
        fa.colmap = s->at<uint16_t>(L.off_colmap);
        fa.rowmap = s->at<uint16_t>(L.off_rowmap);

        kpd::ChunkArgs& c = (*ctab)[j];
        kpd::DetectArgs& d = c.d;
        for (int o = 1; o < L.O; ++o) {
            d.lvl[o] = pyr + L.off_lvl[o];
            d.pitch[o] = L.pitch[o];
        }
        for (int o = 0; o < L.O; ++o) { d.w[o] = L.w[o]; d.h[o] = L.h[o]; }
        d.W = L.W; d.H = L.H; d.O = L.O; d.nc = L.nc; d.nr = L.nr;
        d.sad = fa.sad;
        d.mask = s->at<uint8_t>(L.off_mask);
        d.list_cur = reinterpret_cast<kpd_keypoint*>(s->arena + L.off_sparse + L.clist_stride * (size_t)j);
        d.list_cap = (uint32_t)L.list_cap;
        d.layouts = s->at<kpd::CellLayout>(L.off_layouts);
        d.col_w = s->at<uint16_t>(L.off_colw);
        d.row_h = s->at<uint16_t>(L.off_rowh);
        d.err = s->at<uint32_t>(L.off_hdr) + kHdrErr;
        c.j = j;
        c.Kw = L.Kw;
        c.cell_base = s->at<uint32_t>(L.off_cbase);
        c.marks = s->at<unsigned long long>(L.off_marks);
        c.own_count = s->at<uint32_t>(L.off_own) + (size_t)j * kc;
    }
}

}  // namespace

extern "C" {

int open_stream(int width, int height, const kpd_params* params, void* dev_arena, size_t arena_bytes,
                void* hip_stream, kpd_stream** out)
{
    if (!out) return fail(KPD_EINVAL, "out is NULL");
    *out = nullptr;
    Layout L;
    std::string why;
    if (!make_layout(width, height, params, &L, &why)) return fail(KPD_EINVAL, why);
    if (!dev_arena) return fail(KPD_EINVAL, "arena is NULL");
    if (reinterpret_cast<uintptr_t>(dev_arena) % kAlign) return fail(KPD_EINVAL, "arena not 256-byte aligned");
    if (arena_bytes < L.total)
        return fail(KPD_ENOMEM, "arena has " + std::to_string(arena_bytes) + " bytes, stream needs " +
                                    std::to_string(L.total));
    int dev = 0, lds_max = 0;
    KPD_HIP(hipGetDevice(&dev));
    KPD_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    int group_static = 0;
    KPD_HIP(kpd::group_static_lds(&group_static));
    if (L.lds_bytes > std::max(lds_max, 65536) ||
        std::max(L.glds, L.glds1_512) + group_static > std::max(lds_max, 65536))
        return fail(KPD_EINVAL, "cells need more LDS than a workgroup can hold");
    // a single frame's marked cells run 1024 threads each when one cell fits
    const int det1_threads =
        L.glds1_1024 > 0 && L.glds1_1024 + group_static <= std::max(lds_max, 65536) ? 1024 : 512;
    KPD_HIP(kpd::set_detect_lds_limit(L.lds_bytes));

    kpd_stream* s = new (std::nothrow) kpd_stream();
    if (!s) return fail(KPD_ENOMEM, "host allocation failed");
    s->L = L;
    s->p = *params;
    s->det1_threads = det1_threads;
    s->stream = reinterpret_cast<hipStream_t>(hip_stream);
    s->arena = reinterpret_cast<uint8_t*>(dev_arena);

    // zero the header, both SAD accumulators, the counts and the look-back words
    hipError_t e = hipMemsetAsync(s->arena + L.off_hdr, 0, 64, s->stream);
    for (int k = 0; k < 2 && e == hipSuccess; ++k)
        e = hipMemsetAsync(s->arena + L.off_sad[k], 0, (size_t)L.ncell * 4, s->stream);
    for (int k = 0; k < 2 && e == hipSuccess; ++k)
        e = hipMemsetAsync(s->arena + L.off_count[k], 0, (size_t)L.ncell * 4, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->arena + L.off_status, 0, (size_t)L.ncell * 8, s->stream);
    // constant cell column widths and row heights
    std::vector<uint16_t> colw(L.nc), rowh(L.nr);
    for (int j = 0; j < L.nc; ++j) {
        int a0, a1;
        kpd::cell_span(j, L.nc, L.W, &a0, &a1);
        colw[j] = (uint16_t)(a1 - a0);
    }
    for (int j = 0; j < L.nr; ++j) {
        int a0, a1;
        kpd::cell_span(j, L.nr, L.H, &a0, &a1);
        rowh[j] = (uint16_t)(a1 - a0);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->arena + L.off_colw, colw.data(), colw.size() * 2, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->arena + L.off_rowh, rowh.data(), rowh.size() * 2, hipMemcpyHostToDevice, s->stream);
    std::vector<uint16_t> colmap(L.W), rowmap(L.H);
    for (int x = 0; x < L.W; ++x) colmap[x] = (uint16_t)(((int64_t)x * L.nc) / L.W);
    for (int y = 0; y < L.H; ++y) rowmap[y] = (uint16_t)(((int64_t)y * L.nr) / L.H);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->arena + L.off_colmap, colmap.data(), colmap.size() * 2, hipMemcpyHostToDevice,
                           s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->arena + L.off_rowmap, rowmap.data(), rowmap.size() * 2, hipMemcpyHostToDevice,
                           s->stream);
    std::vector<kpd::CellLayout> layouts(L.ncell);
    for (int c = 0; c < L.ncell; ++c)
        kpd::cell_layout(kpd::cell_rect(c, L.W, L.H, L.nc, L.nr), L.O, L.w, L.h, &layouts[c]);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->arena + L.off_layouts, layouts.data(), layouts.size() * sizeof(kpd::CellLayout),
                           hipMemcpyHostToDevice, s->stream);
    const std::vector<uint32_t> cbase = cell_bases(L);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->arena + L.off_cbase, cbase.data(), cbase.size() * 4, hipMemcpyHostToDevice, s->stream);
    std::vector<uint32_t> pbase(L.ncell);   // per-pixel bases: the decision pixels of the cells before
    uint32_t acc = 0;
    for (int c = 0; c < L.ncell; ++c) {
        pbase[c] = acc;
        acc += (uint32_t)layouts[c].dc_start[L.O];
    }
    if (e == hipSuccess && L.off_pbase)
        e = hipMemcpyAsync(s->arena + L.off_pbase, pbase.data(), pbase.size() * 4, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess && (params->features & KPD_FEAT_DESCRIPTOR))
        e = hipMemcpyAsync(s->arena + L.off_dtab, &desc_tables(), sizeof(kpd::DescTables), hipMemcpyHostToDevice,
                           s->stream);
    std::vector<kpd::ChunkArgs> ctab;
    std::vector<kpd::FrameArgs> ftab;
    if (L.K > 1) {
        if (e == hipSuccess)
            e = hipMemsetAsync(s->arena + L.off_csad, 0, (size_t)L.K * L.ncell * 4, s->stream);
        if (e == hipSuccess) e = hipMemsetAsync(s->arena + L.off_marks, 0, (size_t)L.ncell * L.Kw * 8, s->stream);
        chunk_tables(s, &ctab, &ftab);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->arena + L.off_ctab, ctab.data(), ctab.size() * sizeof(kpd::ChunkArgs),
                               hipMemcpyHostToDevice, s->stream);
        s->chunk_fa = ftab[0];   // later frames' octaves and SAD follow at fixed strides
        int glds = 0;
        group_layouts(L, L.gx, L.gy, L.gthreads / 64, &s->glay, &glds);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->arena + L.off_glay, s->glay.data(), s->glay.size() * sizeof(kpd::GroupLayout),
                               hipMemcpyHostToDevice, s->stream);
    }
    {
        int glds = 0;
        group_layouts(L, 1, 1, kGroupWaves, &s->glay1, &glds);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->arena + L.off_glay1, s->glay1.data(), s->glay1.size() * sizeof(kpd::GroupLayout),
                               hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess)
            e = kpd::set_group_lds_limit(std::max({L.glds, L.glds1_512, glds1_for(L, s->det1_threads)}));
    }
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&s->stage), 64 + kStage * sizeof(kpd_keypoint) + (size_t)L.ncell,
                          hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&s->stage_dev), s->stage, 0);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "open_stream initialisation");
    }
    if (!kpd::handle_add(s)) {
        delete s;
        return fail(KPD_ENOMEM, "host allocation failed");
    }
    *out = s;
    return KPD_OK;
}

int set_thresholds(kpd_stream* s, int32_t fast_t, int32_t id_thresh, uint32_t kb_thresh)
{
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    if (fast_t < 1 || fast_t > 254) return fail(KPD_EINVAL, "fast_t must be in 1..254");
    if (fast_t != s->p.fast_t) s->force_all = true;
    s->p.fast_t = fast_t;
    s->p.id_thresh = id_thresh;
    s->p.kb_thresh = kb_thresh;
    return KPD_OK;
}

}  // extern "C"

namespace {

// Validate and stage the next frame of `s`: copy it into an arena slot when
// asked to, and fill the tick arguments of both passes. The stream state
// advances only in advance_frame, once the work is enqueued.
// Octave o >= 1 is read by the per-pixel mask and so alternates between its
// usual buffer and a second copy, frame by frame.
bool alternates(const kpd_stream* s, int o)
{
    return o >= 1 && ((s->id_mode == 1 && o == s->id_layer) || s->id_mode == 2);
}

uint8_t* alt_level(kpd_stream* s, int o)
{
    return s->arena + s->L.off_lvl_alt + (s->L.off_lvl[o] - s->L.off_lvl[1]);
}

int stage_frame(kpd_stream* s, const uint8_t* frame, size_t pitch_bytes, int flags, kpd::TickArgs* t)
{
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    const Layout& L = s->L;
    if (!frame) return fail(KPD_EINVAL, "frame is NULL");
    if (pitch_bytes < (size_t)L.W || pitch_bytes > (1u << 30)) return fail(KPD_EINVAL, "bad pitch");
    if (flags != KPD_FRAME_HOST && flags != KPD_FRAME_DEVICE && flags != KPD_FRAME_DEVICE_RETAIN)
        return fail(KPD_EINVAL, "bad flags");

    const uint8_t* cur;
    int cur_pitch;
    int cur_dw;
    if (flags == KPD_FRAME_DEVICE_RETAIN) {
        cur = frame;
        cur_pitch = (int)pitch_bytes;
        cur_dw = dword_readable(cur, cur_pitch, L.W, false);
    } else {
        uint8_t* dst = s->at<uint8_t>(L.off_slot[s->cur_slot]);
        const hipMemcpyKind kind = flags == KPD_FRAME_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        if (pitch_bytes <= (size_t)L.slot_pitch) {
            // one linear copy that keeps the caller's pitch: the rows fit the
            // slot, and dword reads past a row's end stay inside it
            KPD_HIP(hipMemcpyAsync(dst, frame, pitch_bytes * (L.H - 1) + L.W, kind, s->stream));
            cur_pitch = (int)pitch_bytes;
            cur_dw = pitch_bytes % 4 == 0 ? 1 : 0;
        } else {
            KPD_HIP(hipMemcpy2DAsync(dst, L.slot_pitch, frame, pitch_bytes, L.W, L.H, kind, s->stream));
            cur_pitch = L.slot_pitch;
            cur_dw = 1;
        }
        cur = dst;
        s->cur_slot ^= 1;
    }

    const uint32_t n = (uint32_t)s->n_pushed;
    const int cur_k = n & 1, prev_k = cur_k ^ 1;       // SAD accumulators go by frame parity
    const int fb_prev = s->fb_last, fb_cur = 1 - s->fb_last;  // keypoint buffers alternate
    const bool all_marked = s->force_all || s->p.id_thresh < 0 || s->p.kb_thresh == 0;
    const bool sad_on = !all_marked && s->p.id_thresh < 255 && s->id_mode == 0;
    // the octaves >= 1 a per-pixel mask reads alternate between two buffers
    // so the previous frame's stay readable
    const int lv = s->id_layer;
    auto level_ptr = [&](int o) -> uint8_t* {
        if (alternates(s, o) && s->layer_buf == 0) return alt_level(s, o);
        return s->at<uint8_t>(L.off_lvl[o]);
    };

    *t = kpd::TickArgs{};
    kpd::FrameArgs& fa = t->f;
    fa.cur = cur;
    fa.cur_pitch = cur_pitch;
    fa.cur_aligned = cur_dw;
    fa.prev = sad_on ? s->prev0 : cur;
    fa.prev_pitch = sad_on ? s->prev_pitch : cur_pitch;
    fa.prev_aligned = sad_on ? s->prev_dw : cur_dw;
    for (int o = 1; o < L.O; ++o) {
        fa.lvl[o] = level_ptr(o);
        fa.pitch[o] = L.pitch[o];
    }
    for (int o = 0; o < L.O; ++o) { fa.w[o] = L.w[o]; fa.h[o] = L.h[o]; }
    fa.W = L.W; fa.H = L.H; fa.O = L.O; fa.nc = L.nc; fa.nr = L.nr;
    fa.tile = L.tile;
    fa.tiles_x = L.tiles_x;
    fa.ntiles = L.tiles_x * L.tiles_y;
    fa.sad_on = sad_on ? 1 : 0;
    fa.sad_slots = L.sad_slots;
    fa.sad_lds_off = kpd::frame_sad_lds_off(L.tile, L.O);
    fa.sad = s->at<uint32_t>(L.off_sad[cur_k]);
    fa.colmap = s->at<uint16_t>(L.off_colmap);
    fa.rowmap = s->at<uint16_t>(L.off_rowmap);
    t->sparse = s->at<kpd_keypoint>(L.off_sparse1);
    t->sparse_base = s->at<uint32_t>(L.off_cbase);
    t->own_count = s->at<uint32_t>(L.off_own1);
    t->glay1 = s->at<kpd::GroupLayout>(L.off_glay1);
    t->al8 = (reinterpret_cast<uintptr_t>(cur) % 8 == 0 && cur_pitch % 8 == 0) ? 1 : 0;
    if (s->p.features & KPD_FEAT_DESCRIPTOR) {
        t->tab = s->at<kpd::DescTables>(L.off_dtab);
        t->desc_prev = s->at<kpd_descriptor>(L.off_desc[fb_prev]);
        t->desc_cur = s->at<kpd_descriptor>(L.off_desc[fb_cur]);
    }
    if (s->p.features & KPD_FEAT_REFINE) {
        t->ref_prev = s->at<kpd_refined>(L.off_ref[fb_prev]);
        t->ref_cur = s->at<kpd_refined>(L.off_ref[fb_cur]);
    }

    kpd::DetectArgs& d = t->d;
    d.lvl[0] = cur;
    d.pitch[0] = cur_pitch;
    for (int o = 1; o < L.O; ++o) {
        d.lvl[o] = level_ptr(o);
        d.pitch[o] = L.pitch[o];
    }
    for (int o = 0; o < L.O; ++o) { d.w[o] = L.w[o]; d.h[o] = L.h[o]; }
    d.lvl0_aligned = cur_dw;
    if (s->id_mode != 0) {
        d.id_mode = s->id_mode;
        d.id_layer = s->id_mode == 1 ? lv : 0;
        // I_{n-1}: level 0 is the previous frame (read only when not every
        // cell is marked), the others the buffers this frame does not write
        d.lprev[0] = s->prev0 ? s->prev0 : cur;
        d.lprev_pitch[0] = s->prev0 ? s->prev_pitch : cur_pitch;
        for (int o = 1; o < L.O; ++o) {
            d.lprev[o] = alternates(s, o) && s->layer_buf == 1 ? alt_level(s, o) : s->at<uint8_t>(L.off_lvl[o]);
            d.lprev_pitch[o] = L.pitch[o];
        }
        d.lds_bits = L.lds_bits;
        d.lds_carr = L.lds_carr;
        d.lds_cwoff = L.lds_cwoff;
        d.lds_cscore = L.lds_cscore;
        d.lds_csrc = L.lds_csrc;
        d.src_cur = s->p.features ? s->at<uint32_t>(L.off_src) : nullptr;
    }
    d.W = L.W; d.H = L.H; d.O = L.O; d.nc = L.nc; d.nr = L.nr;
    d.t = s->p.fast_t;
    d.all_marked = all_marked ? 1 : 0;
    d.id_on = sad_on ? 1 : 0;
    d.id_thresh = s->p.id_thresh;
    d.kb_thresh = s->p.kb_thresh;
    d.sad = s->at<uint32_t>(L.off_sad[cur_k]);
    d.sad_next = s->at<uint32_t>(L.off_sad[prev_k]);
    d.mask = s->at<uint8_t>(L.off_mask);
    d.count_prev = s->at<uint32_t>(L.off_count[fb_prev]);
    d.off_prev = s->at<uint32_t>(L.off_offs[fb_prev]);
    d.list_prev = s->at<kpd_keypoint>(L.off_list[fb_prev]);
    d.count_cur = s->at<uint32_t>(L.off_count[fb_cur]);
    d.off_cur = s->at<uint32_t>(L.off_offs[fb_cur]);
    d.list_cur = s->at<kpd_keypoint>(L.off_list[fb_cur]);
    d.total_cur = s->at<uint32_t>(L.off_hdr) + (fb_cur ? kHdrTotal1 : kHdrTotal0);
    d.list_cap = (uint32_t)L.list_cap1;
    d.layouts = s->at<kpd::CellLayout>(L.off_layouts);
    d.col_w = s->at<uint16_t>(L.off_colw);
    d.row_h = s->at<uint16_t>(L.off_rowh);
    d.status = s->at<unsigned long long>(L.off_status);
    d.epoch = n + 1;
    d.err = s->at<uint32_t>(L.off_hdr) + kHdrErr;

    t->active = 1;
    // the tile pass is skipped when there is neither a pyramid nor a SAD to build
    t->f_on = (L.O > 1 || sad_on) ? 1 : 0;
    return KPD_OK;
}

void advance_frame(kpd_stream* s, const kpd::TickArgs& t)
{
    s->prev0 = t.f.cur;
    s->prev_pitch = t.f.cur_pitch;
    s->prev_dw = t.f.cur_aligned;
    s->force_all = false;
    s->n_pushed += 1;
    s->fb_last = 1 - s->fb_last;
    s->chunk_n = 0;
    if (s->id_mode != 0) s->layer_buf ^= 1;
}

// Copies D_n's per-feature values (one T per feature, in list order) from
// the arena buffers off[0], off[1] that alternate with the keypoint lists.
template <class T>
int copy_features(kpd_stream* s, const size_t* off, T* out, size_t capacity, size_t* count)
{
    if (!count) return fail(KPD_EINVAL, "count is NULL");
    if (s->n_pushed == 0) return fail(KPD_ESTATE, "no frame pushed yet");
    const Layout& L = s->L;
    const int k = s->fb_last;
    uint32_t hdr[4];
    KPD_HIP(hipMemcpyAsync(hdr, s->at<uint32_t>(L.off_hdr), sizeof(hdr), hipMemcpyDeviceToHost, s->stream));
    KPD_HIP(hipStreamSynchronize(s->stream));
    if (hdr[kHdrErr]) return fail(KPD_EDEVICE, "a wait on the device timed out");
    const uint32_t total = std::min<uint32_t>(hdr[k ? kHdrTotal1 : kHdrTotal0], (uint32_t)L.list_cap1);
    *count = total;
    if (total > capacity) return fail(KPD_ETRUNC, "capacity smaller than the feature count");
    if (total > 0) {
        if (!out) return fail(KPD_EINVAL, "out is NULL");
        KPD_HIP(hipMemcpyAsync(out, s->at<T>(off[k]), (size_t)total * sizeof(T), hipMemcpyDeviceToHost, s->stream));
        KPD_HIP(hipStreamSynchronize(s->stream));
    }
    return KPD_OK;
}

// Features of frame i of the last chunk: D_n's for the last frame, else
// the chunk buffer at coff, clist_stride entries apart.
template <class T>
int copy_chunk_features(kpd_stream* s, int i, const size_t* off_last, size_t coff, T* out, size_t capacity,
                        size_t* count)
{
    if (!count) return fail(KPD_EINVAL, "count is NULL");
    if (i < 0 || i >= s->chunk_n) return fail(KPD_EINVAL, "no such frame in the last chunk");
    if (i == s->chunk_n - 1) return copy_features(s, off_last, out, capacity, count);
    const Layout& L = s->L;
    uint32_t hdr[4] = {0, 0, 0, 0}, total = 0;
    KPD_HIP(hipMemcpyAsync(hdr, s->at<uint32_t>(L.off_hdr), sizeof(hdr), hipMemcpyDeviceToHost, s->stream));
    KPD_HIP(hipMemcpyAsync(&total, s->at<uint32_t>(L.off_ctotal) + i, 4, hipMemcpyDeviceToHost, s->stream));
    KPD_HIP(hipStreamSynchronize(s->stream));
    if (hdr[kHdrErr]) return fail(KPD_EDEVICE, "a wait on the device timed out");
    total = std::min<uint32_t>(total, (uint32_t)L.list_cap);
    *count = total;
    if (total > capacity) return fail(KPD_ETRUNC, "capacity smaller than the feature count");
    if (total > 0) {
        if (!out) return fail(KPD_EINVAL, "out is NULL");
        const size_t stride = L.clist_stride / sizeof(kpd_keypoint);
        KPD_HIP(hipMemcpyAsync(out, reinterpret_cast<const T*>(s->arena + coff) + stride * (size_t)i,
                               (size_t)total * sizeof(T), hipMemcpyDeviceToHost, s->stream));
        KPD_HIP(hipStreamSynchronize(s->stream));
    }
    return KPD_OK;
}

}  // namespace

namespace {
std::mutex g_handles_mu;
std::unordered_set<const void*> g_handles;
}  // namespace

namespace kpd {
// error reporting for the other host files of the library
int api_fail(int code, const std::string& msg) { return fail(code, msg); }
int api_hip_fail(hipError_t e, const char* what) { return hip_fail(e, what); }

bool handle_add(const void* h)
{
    try {
        const std::lock_guard<std::mutex> lock(g_handles_mu);
        g_handles.insert(h);
        return true;
    } catch (...) {
        return false;
    }
}

void handle_remove(const void* h)
{
    const std::lock_guard<std::mutex> lock(g_handles_mu);
    g_handles.erase(h);
}

bool handle_live(const void* h)
{
    if (!h) return false;
    const std::lock_guard<std::mutex> lock(g_handles_mu);
    return g_handles.count(h) != 0;
}
}  // namespace kpd

extern "C" {

int push_frame(kpd_stream* s, const uint8_t* frame, size_t pitch_bytes, int flags)
{
    const kpd::TraceRange trace_range("kpd:push_frame");
    kpd::TickArgs t;
    const int rc = stage_frame(s, frame, pitch_bytes, flags, &t);
    if (rc != KPD_OK) return rc;
    const Layout& L = s->L;
    if (t.f_on)
        KPD_HIP(timed(s, KPD_K_FRAME, [&] { return kpd::launch_frame(t.f, s->stream); }));
    if (s->id_mode == 0) {
        // marks and detection of the marked cells (no waits between cells),
        // then D_n by Eq. 1 in one compaction workgroup
        kpd::GroupArgs ga{};
        ga.layouts = s->at<kpd::GroupLayout>(L.off_glay1);
        ga.ngroups = L.ncell;
        ga.nc = L.nc;
        ga.al8 = (reinterpret_cast<uintptr_t>(t.d.lvl[0]) % 8 == 0 && t.d.pitch[0] % 8 == 0) ? 1 : 0;
        const int threads = t.d.all_marked ? 256 : s->det1_threads;
        const int lds = glds1_for(L, threads);
        KPD_HIP(timed(s, KPD_K_DETECT, [&] {
            return kpd::launch_det1_groups(t.d, ga, t.sparse, t.own_count, L.ncell, lds, threads, s->stream);
        }));
        KPD_HIP(timed(s, KPD_K_COMPACT, [&] {
            return kpd::launch_compact1(t.d, t.sparse, t.sparse_base, t.own_count, s->stream);
        }));
    } else {
        const int lds = L.lds_bytes1;
        KPD_HIP(timed(s, KPD_K_DETECT, [&] { return kpd::launch_detect(t.d, L.ncell, lds, s->stream); }));
    }
    if (s->p.features) {
        const int fb_prev = s->fb_last, fb_cur = 1 - s->fb_last;
        kpd::DescArgs da{};
        if (s->p.features & KPD_FEAT_DESCRIPTOR) {
            da.tab = s->at<kpd::DescTables>(L.off_dtab);
            da.desc_prev = s->at<kpd_descriptor>(L.off_desc[fb_prev]);
            da.desc_cur = s->at<kpd_descriptor>(L.off_desc[fb_cur]);
        }
        if (s->p.features & KPD_FEAT_REFINE) {
            da.ref_prev = s->at<kpd_refined>(L.off_ref[fb_prev]);
            da.ref_cur = s->at<kpd_refined>(L.off_ref[fb_cur]);
        }
        for (int o = 0; o < L.O; ++o) {
            da.lvl[o] = t.d.lvl[o];
            da.pitch[o] = t.d.pitch[o];
            da.w[o] = L.w[o];
            da.h[o] = L.h[o];
        }
        da.O = L.O;
        da.t = t.d.t;
        da.mask = t.d.mask;
        da.count_cur = t.d.count_cur;
        da.off_cur = t.d.off_cur;
        da.off_prev = t.d.off_prev;
        da.list_cur = t.d.list_cur;
        da.list_cap = (uint32_t)L.list_cap1;
        da.src_cur = t.d.src_cur;
        KPD_HIP(timed(s, KPD_K_DESCRIBE, [&] { return kpd::launch_describe(da, L.ncell, s->stream); }));
    }
    advance_frame(s, t);
    return KPD_OK;
}

int set_mask_mode(kpd_stream* s, int mode, int layer)
{
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    if (mode < 0 || mode > 2) return fail(KPD_EINVAL, "mode must be 0, 1 or 2");
    if (layer < 0 || layer >= s->L.O) return fail(KPD_EINVAL, "layer must be an octave of the stream");
    if (mode == 2 && layer != 0) return fail(KPD_EINVAL, "mode 2 masks every octave on its own level: layer must be 0");
    if (mode != 0 && !s->p.layer_mask) return fail(KPD_EINVAL, "stream opened without layer_mask");
    if (mode == s->id_mode && (mode != 1 || layer == s->id_layer)) return KPD_OK;
    if (mode != 0 && s->L.lds_bytes1 > 160 * 1024)
        return fail(KPD_EINVAL, "cells too large for a per-pixel mask" +
                                    std::string(s->p.features ? " with features" : "") + " (LDS)");
    if (mode != 0) KPD_HIP(kpd::set_detect_lds_limit(s->L.lds_bytes1));
    s->id_mode = mode;
    s->id_layer = mode == 1 ? layer : 0;
    s->layer_buf = 0;
    s->force_all = true;   // the previous frame's layer may not be kept: re-detect every cell once
    return KPD_OK;
}

// Frames per workgroup of the sequential tile pass of a chunk of n frames
// (0 when the stream's tiles cannot take it). Every workgroup of a chunk
// does the same work, so the pass takes as long as its rounds of `cap`
// resident workgroups: the run is chosen for the fullest last round over
// one to four rounds, at least 8 frames a run (each run re-reads the frame
// before it) and a multiple of four (the kernel's steps go in fours).
int seq_run(const Layout& L, int n, int cap)
{
    if (!L.seq_ok || cap <= 0) return 0;
    const int ntiles = L.seq_ntiles;
    int best = 0;
    double best_eff = 0.0;
    for (int m = 1; m <= 4; ++m) {
        const int nruns = std::max(1, m * cap / ntiles);
        const int run = (std::max(6, (n + nruns - 1) / nruns) + 3) / 4 * 4;   // whole groups of four steps
        const int used = (n + run - 1) / run;
        const int rounds = (used * ntiles + cap - 1) / cap;
        const double eff = (double)used * ntiles / ((double)rounds * cap);
        if (eff > best_eff + 1e-9) {
            best_eff = eff;
            best = run;
        }
    }
    best = std::min(best, n);
    if (kpd::frame_seq_lds_bytes(L.seq_slots, best) > 65536) return 0;
    return best;
}

int push_frames(kpd_stream* s, const uint8_t* frames, size_t frame_stride, size_t pitch_bytes, int n_frames)
{
    const kpd::TraceRange trace_range("kpd:push_frames");
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    const Layout& L = s->L;
    if (L.K < 2) return fail(KPD_EINVAL, "stream opened without chunk_frames");
    // per-pixel masks (Sec. 3.1): their marks come from pixels alone, so T_H
    // (whose marks chain through the counts frame by frame) must be off
    const bool pixel = s->id_mode != 0;
    if (pixel && s->p.kb_thresh != KPD_KB_OFF && s->p.kb_thresh != 0 && s->p.id_thresh >= 0)
        return fail(KPD_EINVAL, "the layer mask in chunks needs kb_thresh off");
    if (pixel && L.pm_lds > 60 * 1024) return fail(KPD_EINVAL, "cells too large for the layer mask in chunks");
    if (pixel && s->p.features && L.list_cap >= (1u << kpd::kPixelFrameShift))
        return fail(KPD_EINVAL, "frame too large for features with a per-pixel mask in chunks");
    if (!frames) return fail(KPD_EINVAL, "frames is NULL");
    if (n_frames < 1 || n_frames > L.K) return fail(KPD_EINVAL, "n_frames out of range");
    if (pitch_bytes < (size_t)L.W || pitch_bytes > (1u << 30)) return fail(KPD_EINVAL, "bad pitch");
    if (n_frames > 1 && frame_stride < pitch_bytes * (size_t)(L.H - 1) + (size_t)L.W)
        return fail(KPD_EINVAL, "frames overlap");
    const int pitch = (int)pitch_bytes;
    const uint32_t n0 = (uint32_t)s->n_pushed;
    const int fb_prev = s->fb_last, fb_next = 1 - s->fb_last;
    kpd::ChunkHead h{};
    h.frames = frames;
    h.stride = frame_stride;
    h.pitch = pitch;
    h.aligned = dword_readable(frames, pitch, L.W, false) && frame_stride % 4 == 0;
    h.prev0 = s->prev0 ? s->prev0 : frames;   // read only when frame 0 tests intensity differences
    h.prev0_pitch = s->prev0 ? s->prev_pitch : pitch;
    h.prev0_aligned = s->prev0 ? s->prev_dw : h.aligned;
    h.n_frames = n_frames;
    h.force0 = s->force_all ? 1 : 0;
    h.all_marked = (s->p.id_thresh < 0 || s->p.kb_thresh == 0) ? 1 : 0;
    h.t = s->p.fast_t;
    h.id_thresh = s->p.id_thresh;
    h.kb_thresh = s->p.kb_thresh;
    // marks read the previous frame's counts only when T_H can mark a cell
    // and the parameters do not mark every cell anyway
    h.kb_chain = (s->p.kb_thresh != KPD_KB_OFF && !h.all_marked) ? 1 : 0;
    h.prev_count = s->at<uint32_t>(L.off_count[fb_prev]);
    h.ntiles = L.ctiles_x * L.ctiles_y;
    h.ncell = L.ncell;
    h.nc = L.nc;
    h.sad0 = s->at<uint32_t>(L.off_csad);
    h.col_w = s->at<uint16_t>(L.off_colw);
    h.row_h = s->at<uint16_t>(L.off_rowh);
    h.marks = s->at<unsigned long long>(L.off_marks);
    h.mask = s->at<uint8_t>(L.off_mask);
    h.Kw = L.Kw;
    h.work = s->at<uint32_t>(L.off_work);
    h.work_count = s->at<uint32_t>(L.off_hdr) + kHdrWork;
    // the tile pass is needed for coarser octaves or intensity differences
    // (per-cell ones: the per-pixel masks read the octaves it writes)
    const bool any_tiles = L.O > 1 || (!pixel && s->p.id_thresh >= 0 && s->p.id_thresh < 255 && !h.all_marked &&
                                       (n_frames > 1 || !h.force0));
    const kpd::ChunkArgs* ctab = s->at<kpd::ChunkArgs>(L.off_ctab);
    // frames that test intensity differences walk each tile in frame order
    // (each frame read once) when the tile builds its octaves in registers
    // (16-byte aligned rows of the chunk's frames and of the frame before)
    auto al16 = [](const uint8_t* p, size_t pitch_b) {
        return reinterpret_cast<uintptr_t>(p) % 16 == 0 && pitch_b % 16 == 0;
    };
    if (L.seq_ok && s->seq_cap == 0) {
        // resident workgroups of the sequential pass (its LDS is a few KB)
        int cap = 0;
        KPD_HIP(kpd::frame_seq_capacity(kpd::frame_seq_lds_bytes(L.seq_slots, 64), &cap));
        s->seq_cap = std::max(cap, 1);
    }
    const int run = seq_run(L, n_frames, s->seq_cap);
    const bool seq = run > 0 && !pixel && s->p.id_thresh >= 0 && s->p.id_thresh < 255 && !h.all_marked &&
                     (n_frames > 1 || !h.force0) && al16(frames, pitch_bytes) && frame_stride % 16 == 0 &&
                     (h.force0 || al16(h.prev0, (size_t)h.prev0_pitch));
    // the layers of the frame before the chunk that a per-pixel mask reads:
    // kept in the second octave buffer (octave buffer 0 is chunk frame 0's)
    const bool pixel_diff = pixel && !h.all_marked;
    if (pixel_diff && !h.force0 && L.O > 1 && s->layer_buf == 0)
        KPD_HIP(hipMemcpyAsync(s->arena + L.off_lvl_alt, s->arena + L.off_lvl[1], L.pyr_stride,
                               hipMemcpyDeviceToDevice, s->stream));
    kpd::ChunkHead ht = h;
    if (pixel) ht.id_thresh = 255;   // no per-cell differences in the tile pass
    if (any_tiles)
        KPD_HIP(timed(s, KPD_K_FRAME, [&] {
            if (seq) {
                // chunks above the 256 MB last level cache stream their frames
                const bool nt = (double)n_frames * (double)frame_stride > 256.0 * 1024 * 1024;
                const kpd::SeqGrid g{L.seq_tile_w, L.seq_tiles_x, L.seq_ntiles, L.seq_slots, run};
                return kpd::launch_frame_chunk_seq(s->chunk_fa, L.pyr_stride, h, g, nt, s->stream);
            }
            return kpd::launch_frame_chunk(s->chunk_fa, L.pyr_stride, ht,
                                           kpd::frame_lds_bytes(L.ctile, L.O, L.csad_slots), s->stream);
        }));
    kpd::PixelChunkArgs pa{};
    if (h.all_marked) {
        // every cell of every frame: one workgroup per (frame, cell)
        kpd::GroupArgs ga{};
        ga.layouts = s->at<kpd::GroupLayout>(L.off_glay);
        ga.ngroups = L.ngroups;
        ga.nc = L.nc;
        ga.al8 = (reinterpret_cast<uintptr_t>(frames) % 8 == 0 && frame_stride % 8 == 0 && pitch % 8 == 0) ? 1 : 0;
        KPD_HIP(timed(s, KPD_K_DETECT, [&] {
            return kpd::launch_detect_chunk_groups(ctab, h, ga, L.glds, L.gthreads, s->stream);
        }));
    } else {
        // listed (frame, cell) items, each detected with its one-cell layout
        kpd::GroupArgs g1{};
        g1.layouts = s->at<kpd::GroupLayout>(L.off_glay1);
        g1.ngroups = L.ncell;
        g1.nc = L.nc;
        g1.al8 = (reinterpret_cast<uintptr_t>(frames) % 8 == 0 && frame_stride % 8 == 0 && pitch % 8 == 0) ? 1 : 0;
        auto detect = [&](int round) {
            return timed(s, KPD_K_DETECT, [&] {
                const int nt = list_threads(L);
                return kpd::launch_detect_list_groups(ctab, h, g1, glds1_for(L, nt), nt, round, s->stream);
            });
        };
        if (pixel_diff) {
            pa.table = ctab;
            pa.frames = frames;
            pa.stride = frame_stride;
            pa.pitch = pitch;
            pa.prev_lvl[0] = h.prev0;
            pa.prev_pitch[0] = h.prev0_pitch;
            for (int o = 1; o < L.O; ++o) {
                pa.prev_lvl[o] = alt_level(s, o);
                pa.prev_pitch[o] = L.pitch[o];
            }
            pa.n_frames = n_frames;
            pa.ncell = L.ncell;
            pa.nc = L.nc;
            pa.nr = L.nr;
            pa.W = L.W;
            pa.H = L.H;
            pa.O = L.O;
            pa.Kw = L.Kw;
            pa.one = s->id_mode == 1 ? 1 : 0;
            pa.l_lo = s->id_mode == 1 ? s->id_layer : 0;
            pa.l_hi = s->id_mode == 1 ? s->id_layer : L.O - 1;
            pa.id_thresh = s->p.id_thresh;
            pa.force0 = h.force0;
            pa.flags = s->at<uint32_t>(L.off_pflag);
            pa.fp = s->at<unsigned long long>(L.off_fp);
            pa.fpw = L.fpw;
            pa.marks = h.marks;
            pa.layouts = s->at<kpd::CellLayout>(L.off_layouts);
            pa.cell_base = s->at<uint32_t>(L.off_cbase);
            pa.list_cap = (uint32_t)L.list_cap;
            pa.sparse = reinterpret_cast<const kpd_keypoint*>(s->arena + L.off_sparse);
            pa.own = s->at<uint32_t>(L.off_own);
            pa.pbase = s->at<uint32_t>(L.off_pbase);
            pa.merged = reinterpret_cast<kpd_keypoint*>(s->arena + L.off_msparse);
            pa.mcount = s->at<uint32_t>(L.off_mcount);
            pa.list_stride = L.clist_stride / sizeof(kpd_keypoint);
            pa.plist_cap = (uint32_t)L.list_cap1;
            pa.prev_list = s->at<kpd_keypoint>(L.off_list[fb_prev]);
            pa.prev_count = s->at<uint32_t>(L.off_count[fb_prev]);
            pa.prev_offs = s->at<uint32_t>(L.off_offs[fb_prev]);
            pa.prev_cap = (uint32_t)L.list_cap1;
            pa.lds_pres = L.pm_pres;
            pa.lds_score = L.pm_score;
            pa.lds_fp = L.pm_fp;
            pa.lds_ents = L.pm_ents;
            pa.lds_tgate = L.pm_tgate;
            pa.lds_txy = L.pm_txy;
            pa.lds_toct = L.pm_toct;
            pa.tab_on = L.pm_tab;
            pa.lds_tsrc = L.pm_tsrc;
            pa.lds_bytes = L.pm_lds;
            if (s->p.features) {
                pa.msrc = s->at<uint32_t>(L.off_msrc);
                pa.t = s->p.fast_t;
                pa.counts = s->at<uint32_t>(L.off_ccount);
                pa.offs = s->at<uint32_t>(L.off_coffs);
                pa.last_count = s->at<uint32_t>(L.off_count[fb_next]);
                pa.last_offs = s->at<uint32_t>(L.off_offs[fb_next]);
                pa.dlist_cap = (uint32_t)L.list_cap1;
                if (s->p.features & KPD_FEAT_DESCRIPTOR) {
                    pa.tab = s->at<kpd::DescTables>(L.off_dtab);
                    pa.sdesc = s->at<kpd_descriptor>(L.off_sdesc);
                    pa.cdesc = reinterpret_cast<kpd_descriptor*>(s->arena + L.off_cdesc);
                    pa.last_desc = s->at<kpd_descriptor>(L.off_desc[fb_next]);
                    pa.prev_desc = s->at<kpd_descriptor>(L.off_desc[fb_prev]);
                }
                if (s->p.features & KPD_FEAT_REFINE) {
                    pa.sref = s->at<kpd_refined>(L.off_sref);
                    pa.cref = reinterpret_cast<kpd_refined*>(s->arena + L.off_cref);
                    pa.last_ref = s->at<kpd_refined>(L.off_ref[fb_next]);
                    pa.prev_ref = s->at<kpd_refined>(L.off_ref[fb_prev]);
                }
            }
            pa.batch = L.pm_batch;
            pa.ents_cap = kPixelStagedMaxima;
        }
        if (pixel_diff) {
            // changed mask pixels, marks of the cells with one, detection of
            // those cells, then Eq. 1 per feature along each cell's frames
            kpd::ChunkHead hm = h;
            hm.sad0 = pa.flags;
            hm.id_thresh = 0;   // a cell is marked when its change flag is above 0
            KPD_HIP(timed(s, KPD_K_MARK, [&] { return kpd::launch_pixel_diff_chunk(pa, s->stream); }));
            if (s->id_layer == 0) {
                // masks on level 0 (mode 2, or mode 1 on layer 0): pixel noise
                // lists nearly every (frame, cell), so every cell of every
                // frame is detected by the full-frame group detector, and the
                // mark pass then replaces the mark words it sets (the merge
                // reads only the listed frames' maxima)
                kpd::GroupArgs ga{};
                ga.layouts = s->at<kpd::GroupLayout>(L.off_glay);
                ga.ngroups = L.ngroups;
                ga.nc = L.nc;
                ga.al8 = g1.al8;
                KPD_HIP(timed(s, KPD_K_DETECT, [&] {
                    return kpd::launch_detect_chunk_groups(ctab, h, ga, L.glds, L.gthreads, s->stream);
                }));
                KPD_HIP(timed(s, KPD_K_MARK, [&] { return kpd::launch_mark_chunk(hm, s->stream); }));
            } else {
                KPD_HIP(timed(s, KPD_K_MARK, [&] { return kpd::launch_mark_chunk(hm, s->stream); }));
                KPD_HIP(detect(0));
            }
            KPD_HIP(timed(s, KPD_K_MARK, [&] { return kpd::launch_pixel_merge_chunk(pa, s->stream); }));
            if (s->p.features)   // the listed frames' maxima, on their frames' levels
                KPD_HIP(timed(s, KPD_K_DESCRIBE, [&] { return kpd::launch_pixel_features_chunk(pa, s->stream); }));
        } else if (h.kb_chain) {
            // marks that depend on the counts: detect every frame a cell's
            // chain can mark, then walk each cell's frames to keep the marks
            const uint32_t* own = s->at<uint32_t>(L.off_own);
            KPD_HIP(timed(s, KPD_K_MARK, [&] { return kpd::launch_spec_chunk(h, s->stream); }));
            KPD_HIP(detect(0));
            KPD_HIP(timed(s, KPD_K_MARK, [&] { return kpd::launch_spec2_chunk(h, own, s->stream); }));
            KPD_HIP(detect(1));
            KPD_HIP(timed(s, KPD_K_MARK, [&] { return kpd::launch_resolve_chunk(h, own, s->stream); }));
        } else {
            // marks from the SAD alone: list the marked cells, detect only those
            KPD_HIP(timed(s, KPD_K_MARK, [&] { return kpd::launch_mark_chunk(h, s->stream); }));
            KPD_HIP(detect(0));
        }
    }
    kpd::CompactArgs ca{};
    ca.ncell = L.ncell;
    ca.last = n_frames - 1;
    ca.Kw = L.Kw;
    ca.list_cap = (uint32_t)L.list_cap;
    ca.list_stride = L.clist_stride / sizeof(kpd_keypoint);
    ca.sparse = reinterpret_cast<const kpd_keypoint*>(s->arena + L.off_sparse);
    ca.cell_base = s->at<uint32_t>(L.off_cbase);
    ca.marks = s->at<unsigned long long>(L.off_marks);
    ca.own_count = s->at<uint32_t>(L.off_own);
    ca.prev_list = s->at<kpd_keypoint>(L.off_list[fb_prev]);
    ca.prev_count = s->at<uint32_t>(L.off_count[fb_prev]);
    ca.prev_offs = s->at<uint32_t>(L.off_offs[fb_prev]);
    ca.lists = reinterpret_cast<kpd_keypoint*>(s->arena + L.off_clist);
    ca.counts = s->at<uint32_t>(L.off_ccount);
    ca.offs = s->at<uint32_t>(L.off_coffs);
    ca.totals = s->at<uint32_t>(L.off_ctotal);
    ca.next_list = s->at<kpd_keypoint>(L.off_list[fb_next]);
    ca.next_count = s->at<uint32_t>(L.off_count[fb_next]);
    ca.next_offs = s->at<uint32_t>(L.off_offs[fb_next]);
    ca.next_total = s->at<uint32_t>(L.off_hdr) + (fb_next ? kHdrTotal1 : kHdrTotal0);
    ca.sad_chunk = s->at<uint32_t>(L.off_csad);
    const uint32_t n_last = n0 + (uint32_t)n_frames - 1;
    ca.sad_stats = s->at<uint32_t>(L.off_sad[n_last & 1]);
    ca.sad_single_next = s->at<uint32_t>(L.off_sad[(n_last + 1) & 1]);
    ca.work_count = h.work_count;
    if (pixel_diff) {
        // the merged lists: one entry per decision pixel at most
        ca.sparse = pa.merged;
        ca.cell_base = pa.pbase;
        ca.own_count = pa.mcount;
        ca.list_cap = (uint32_t)L.list_cap1;
    }
    KPD_HIP(timed(s, KPD_K_COMPACT, [&] { return kpd::launch_compact_chunk(ca, n_frames, s->stream); }));
    if (s->p.features && pixel_diff) {
        // each frame's records from the sources the merge kept
        KPD_HIP(timed(s, KPD_K_DESCRIBE, [&] { return kpd::launch_pixel_gather_chunk(pa, s->stream); }));
    } else if (s->p.features) {
        // features of every frame's list: computed where a frame marked a
        // cell, carried with the keypoints elsewhere (Eq. 1)
        kpd::DescChunkArgs da{};
        da.table = ctab;
        da.frames = frames;
        da.stride = frame_stride;
        da.pitch = pitch;
        da.n_frames = n_frames;
        da.ncell = L.ncell;
        da.Kw = L.Kw;
        da.O = L.O;
        da.t = s->p.fast_t;
        da.marks = ca.marks;
        da.list_cap = ca.list_cap;
        da.list_stride = ca.list_stride;
        da.lists = ca.lists;
        da.counts = ca.counts;
        da.offs = ca.offs;
        da.last_list = ca.next_list;
        da.last_count = ca.next_count;
        da.last_offs = ca.next_offs;
        da.prev_offs = ca.prev_offs;
        if (s->p.features & KPD_FEAT_DESCRIPTOR) {
            da.tab = s->at<kpd::DescTables>(L.off_dtab);
            da.descs = reinterpret_cast<kpd_descriptor*>(s->arena + L.off_cdesc);
            da.last_desc = s->at<kpd_descriptor>(L.off_desc[fb_next]);
            da.prev_desc = s->at<kpd_descriptor>(L.off_desc[fb_prev]);
        }
        if (s->p.features & KPD_FEAT_REFINE) {
            da.refs = reinterpret_cast<kpd_refined*>(s->arena + L.off_cref);
            da.last_ref = s->at<kpd_refined>(L.off_ref[fb_next]);
            da.prev_ref = s->at<kpd_refined>(L.off_ref[fb_prev]);
        }
        KPD_HIP(timed(s, KPD_K_DESCRIBE, [&] { return kpd::launch_describe_chunk(da, s->stream); }));
    }

    const uint8_t* last = frames + (size_t)(n_frames - 1) * frame_stride;
    s->prev0 = last;
    s->prev_pitch = pitch;
    s->prev_dw = dword_readable(last, pitch, L.W, false);
    if (pixel && L.O > 1) {
        // the last frame's octaves are I_{n-1}'s for the next push: octave
        // buffer 0 holds them after a one-frame chunk, else they go to the
        // second buffer
        if (n_frames > 1) {
            KPD_HIP(hipMemcpyAsync(s->arena + L.off_lvl_alt, s->arena + L.off_lvl[1] + L.pyr_stride * (n_frames - 1),
                                   L.pyr_stride, hipMemcpyDeviceToDevice, s->stream));
            s->layer_buf = 1;
        } else {
            s->layer_buf = 0;
        }
    }
    s->force_all = false;
    s->n_pushed += n_frames;
    s->fb_last = fb_next;
    s->chunk_n = n_frames;
    return KPD_OK;
}

int kpd_chunk_result(kpd_stream* s, int i, const kpd_keypoint** d_list, const uint32_t** d_count)
{
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    if (i < 0 || i >= s->chunk_n) return fail(KPD_EINVAL, "no such frame in the last chunk");
    const Layout& L = s->L;
    if (i == s->chunk_n - 1) return kpd_device_result(s, d_list, d_count);   // the last frame's D is D_n
    if (d_list) *d_list = reinterpret_cast<const kpd_keypoint*>(s->arena + L.off_clist + L.clist_stride * (size_t)i);
    if (d_count) *d_count = s->at<uint32_t>(L.off_ctotal) + i;
    return KPD_OK;
}

int get_chunk_keypoints(kpd_stream* s, int i, kpd_keypoint* out, size_t capacity, size_t* count)
{
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    if (!count) return fail(KPD_EINVAL, "count is NULL");
    if (i < 0 || i >= s->chunk_n) return fail(KPD_EINVAL, "no such frame in the last chunk");
    if (i == s->chunk_n - 1) return get_keypoints(s, out, capacity, count, nullptr);   // D_n itself
    const Layout& L = s->L;
    uint32_t hdr[4] = {0, 0, 0, 0}, total = 0;
    KPD_HIP(hipMemcpyAsync(hdr, s->at<uint32_t>(L.off_hdr), sizeof(hdr), hipMemcpyDeviceToHost, s->stream));
    KPD_HIP(hipMemcpyAsync(&total, s->at<uint32_t>(L.off_ctotal) + i, 4, hipMemcpyDeviceToHost, s->stream));
    KPD_HIP(hipStreamSynchronize(s->stream));
    if (hdr[kHdrErr]) return fail(KPD_EDEVICE, "a wait on the device timed out");
    *count = total;
    if (total > capacity) return fail(KPD_ETRUNC, "capacity smaller than the keypoint count");
    if (total > 0) {
        if (!out) return fail(KPD_EINVAL, "out is NULL");
        KPD_HIP(hipMemcpyAsync(out, s->arena + L.off_clist + L.clist_stride * (size_t)i,
                               (size_t)total * sizeof(kpd_keypoint), hipMemcpyDeviceToHost, s->stream));
        KPD_HIP(hipStreamSynchronize(s->stream));
    }
    return KPD_OK;
}

int get_keypoints(kpd_stream* s, kpd_keypoint* out, size_t capacity, size_t* count, uint8_t* cell_mask)
{
    const kpd::TraceRange trace_range("kpd:get_keypoints");
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    if (!count) return fail(KPD_EINVAL, "count is NULL");
    if (s->n_pushed == 0) return fail(KPD_ESTATE, "no frame pushed yet");
    const Layout& L = s->L;
    const int k = s->fb_last;
    // one round trip: a kernel writes the header, the first entries of D_n
    // and the mask into the pinned staging buffer
    const size_t pre = std::min(L.list_cap1, kStage);
    uint8_t* st_list = s->stage + 64;
    uint8_t* st_mask = st_list + kStage * sizeof(kpd_keypoint);
    KPD_HIP(kpd::launch_publish(s->at<uint32_t>(L.off_hdr), k ? kHdrTotal1 : kHdrTotal0,
                                s->at<kpd_keypoint>(L.off_list[k]), (uint32_t)pre,
                                cell_mask ? s->at<uint8_t>(L.off_mask) : nullptr, L.ncell, (uint32_t)kStage,
                                s->stage_dev, s->stream));
    KPD_HIP(hipStreamSynchronize(s->stream));
    uint32_t hdr[4];
    std::memcpy(hdr, s->stage, sizeof(hdr));
    if (hdr[kHdrErr]) return fail(KPD_EDEVICE, "a wait on the device timed out");
    const uint32_t total = hdr[k ? kHdrTotal1 : kHdrTotal0];
    *count = total;
    if (total > capacity) return fail(KPD_ETRUNC, "capacity smaller than the keypoint count");
    if (total > 0) {
        if (!out) return fail(KPD_EINVAL, "out is NULL");
        const size_t first = std::min<size_t>(total, pre);
        std::memcpy(out, st_list, first * sizeof(kpd_keypoint));
        if (total > first) {
            KPD_HIP(hipMemcpyAsync(out + first, s->at<kpd_keypoint>(L.off_list[k]) + first,
                                   (size_t)(total - first) * sizeof(kpd_keypoint), hipMemcpyDeviceToHost, s->stream));
            KPD_HIP(hipStreamSynchronize(s->stream));
        }
    }
    if (cell_mask) std::memcpy(cell_mask, st_mask, (size_t)L.ncell);
    return KPD_OK;
}

int get_descriptors(kpd_stream* s, kpd_descriptor* out, size_t capacity, size_t* count)
{
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    if (!(s->p.features & KPD_FEAT_DESCRIPTOR)) return fail(KPD_EINVAL, "stream opened without descriptors");
    return copy_features(s, s->L.off_desc, out, capacity, count);
}

int get_refined(kpd_stream* s, kpd_refined* out, size_t capacity, size_t* count)
{
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    if (!(s->p.features & KPD_FEAT_REFINE)) return fail(KPD_EINVAL, "stream opened without refinement");
    return copy_features(s, s->L.off_ref, out, capacity, count);
}

int get_chunk_descriptors(kpd_stream* s, int i, kpd_descriptor* out, size_t capacity, size_t* count)
{
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    if (!(s->p.features & KPD_FEAT_DESCRIPTOR)) return fail(KPD_EINVAL, "stream opened without descriptors");
    return copy_chunk_features(s, i, s->L.off_desc, s->L.off_cdesc, out, capacity, count);
}

int get_chunk_refined(kpd_stream* s, int i, kpd_refined* out, size_t capacity, size_t* count)
{
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    if (!(s->p.features & KPD_FEAT_REFINE)) return fail(KPD_EINVAL, "stream opened without refinement");
    return copy_chunk_features(s, i, s->L.off_ref, s->L.off_cref, out, capacity, count);
}

int kpd_desc_point(int sector, int i, int* dx, int* dy)
{
    if (sector < 0 || sector >= kpd::kDescSectors || i < 0 || i >= kpd::kDescPts || !dx || !dy) return -1;
    const kpd::DescTables& T = desc_tables();
    *dx = T.pt[sector][i][0];
    *dy = T.pt[sector][i][1];
    return T.half[i];
}

int close_stream(kpd_stream* s)
{
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    if (s->batch) {   // leave the batch first, so that it holds no released stream
        const int rc = batch_detach(s->batch, s);
        if (rc != KPD_OK) return rc;
    }
    hipError_t e = hipStreamSynchronize(s->stream);
    kpd::handle_remove(s);
    delete s;
    if (e != hipSuccess) return hip_fail(e, "close_stream");
    return KPD_OK;
}

int reset_stream(kpd_stream* s)
{
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    s->force_all = true;
    return KPD_OK;
}

int kpd_profile(kpd_stream* s, int enable)
{
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    s->timer.on = enable != 0;
    return KPD_OK;
}

int kpd_profile_read(kpd_stream* s, double* ms, uint64_t* launches)
{
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    KPD_HIP(hipStreamSynchronize(s->stream));
    for (auto& p : s->timer.pending) {
        float t = 0.f;
        KPD_HIP(hipEventElapsedTime(&t, p.second.first, p.second.second));
        s->timer.ms[p.first] += t;
        s->timer.launches[p.first] += 1;
        s->timer.free_events.push_back(p.second.first);
        s->timer.free_events.push_back(p.second.second);
    }
    s->timer.pending.clear();
    for (int k = 0; k < KPD_NKERNELS; ++k) {
        if (ms) ms[k] = s->timer.ms[k];
        if (launches) launches[k] = s->timer.launches[k];
        s->timer.ms[k] = 0;
        s->timer.launches[k] = 0;
    }
    return KPD_OK;
}

int kpd_device_result(kpd_stream* s, const kpd_keypoint** d_list, const uint32_t** d_count)
{
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    if (s->n_pushed == 0) return fail(KPD_ESTATE, "no frame pushed yet");
    const int k = s->fb_last;
    if (d_list) *d_list = s->at<kpd_keypoint>(s->L.off_list[k]);
    if (d_count) *d_count = s->at<uint32_t>(s->L.off_hdr) + (k ? kHdrTotal1 : kHdrTotal0);
    return KPD_OK;
}

int kpd_cell_stats(kpd_stream* s, uint32_t* sad, uint32_t* counts)
{
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    if (s->n_pushed == 0) return fail(KPD_ESTATE, "no frame pushed yet");
    const int k = (s->n_pushed - 1) & 1;
    const size_t n = (size_t)s->L.ncell * 4;
    if (sad) KPD_HIP(hipMemcpyAsync(sad, s->at<uint32_t>(s->L.off_sad[k]), n, hipMemcpyDeviceToHost, s->stream));
    if (counts)
        KPD_HIP(hipMemcpyAsync(counts, s->at<uint32_t>(s->L.off_count[s->fb_last]), n, hipMemcpyDeviceToHost,
                               s->stream));
    KPD_HIP(hipStreamSynchronize(s->stream));
    return KPD_OK;
}

// ---------------------------------------------------------------- batching

}  // extern "C"

struct kpd_batch {
    hipStream_t stream = nullptr;
    int max_streams = 0, max_blocks = 0;
    bool use_graph = true;
    uint8_t* scratch = nullptr;
    kpd::TickArgs* dev_table[2] = {nullptr, nullptr};
    uint16_t* dev_fmap = nullptr;
    uint16_t* dev_cmap = nullptr;
    uint32_t* dev_work = nullptr;         // marked cells of a tick (global cell indices)
    uint32_t* dev_work_count = nullptr;   // their number, cleared by the compaction pass
    kpd::TickArgs* host_table[2] = {nullptr, nullptr};  // pinned
    hipEvent_t table_free[2] = {nullptr, nullptr};      // upload of host_table[k] done
    bool table_used[2] = {false, false};
    std::vector<kpd_stream*> streams;
    std::vector<kpd::TickArgs> staged;                  // per attached stream
    std::vector<char> has_frame;
    int frame_blocks = 0, cell_blocks = 0;
    int frame_lds = 16, detect_lds = 16, detect_glds = 16;
    // the single-launch tick: its counters, LDS and grid (0 when it cannot
    // run: the device holds too few of its workgroups at once)
    bool single_launch = false;
    kpd::TickSync* dev_sync = nullptr;
    int tick_lds = 16, tick_grid = 0;
    bool features = false;   // an attached stream computes descriptors or refined values
    bool pixel = false;      // an attached stream may run a per-pixel mask (opened with layer_mask)
    int pixel_lds = 16;      // the per-pixel cell pass's LDS
    bool maps_dirty = true;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    uint64_t ticks = 0;
};

namespace {

// Batch scratch: two tick tables, the workgroup -> stream maps of the tile
// and cell passes, the work list of marked cells and its counter.
size_t batch_layout(int max_streams, int max_blocks, size_t* off_table, size_t* off_fmap, size_t* off_cmap,
                    size_t* off_work = nullptr, size_t* off_sync = nullptr)
{
    size_t off = 0;
    off_table[0] = off; off = align_up(off + (size_t)max_streams * sizeof(kpd::TickArgs));
    off_table[1] = off; off = align_up(off + (size_t)max_streams * sizeof(kpd::TickArgs));
    *off_fmap = off; off = align_up(off + (size_t)max_blocks * 2);
    *off_cmap = off; off = align_up(off + (size_t)max_blocks * 2);
    if (off_work) *off_work = off;
    off = align_up(off + 256 + (size_t)max_blocks * 4);   // counter, then the list
    if (off_sync) *off_sync = off;
    off = align_up(off + sizeof(kpd::TickSync));
    return off;
}

void drop_graphs(kpd_batch* b)
{
    for (int k = 0; k < 2; ++k)
        if (b->graph[k]) { (void)hipGraphExecDestroy(b->graph[k]); b->graph[k] = nullptr; }
}

// Rebuild the workgroup -> stream maps after the attached set changed.
int rebuild_maps(kpd_batch* b)
{
    std::vector<uint16_t> fmap, cmap;
    int fl = 16, dl = 16, gl = 16;
    bool feats = false, pix = false;
    int pl = 16;
    for (size_t i = 0; i < b->streams.size(); ++i) {
        const Layout& L = b->streams[i]->L;
        feats = feats || b->streams[i]->p.features != 0;
        if (b->streams[i]->p.layer_mask) {
            pix = true;
            pl = std::max(pl, L.lds_bytes1);
        }
        const int nt = L.tiles_x * L.tiles_y;
        fmap.insert(fmap.end(), (size_t)nt, (uint16_t)i);
        cmap.insert(cmap.end(), (size_t)L.ncell, (uint16_t)i);
        fl = std::max(fl, kpd::frame_lds_bytes(L.tile, L.O, L.sad_slots));
        dl = std::max(dl, L.lds_bytes);
        gl = std::max(gl, L.glds1_256);
    }
    if ((int)fmap.size() > b->max_blocks || (int)cmap.size() > b->max_blocks)
        return fail(KPD_ENOMEM, "batch workgroup capacity exceeded");
    KPD_HIP(hipStreamSynchronize(b->stream));  // no tick in flight reads the old maps
    if (!fmap.empty()) KPD_HIP(hipMemcpy(b->dev_fmap, fmap.data(), fmap.size() * 2, hipMemcpyHostToDevice));
    if (!cmap.empty()) KPD_HIP(hipMemcpy(b->dev_cmap, cmap.data(), cmap.size() * 2, hipMemcpyHostToDevice));
    KPD_HIP(kpd::set_detect_lds_limit(std::max(dl, pl)));
    b->frame_blocks = (int)fmap.size();
    b->cell_blocks = (int)cmap.size();
    b->frame_lds = fl;
    b->detect_lds = dl;
    b->detect_glds = gl;
    b->features = feats;
    b->pixel = pix;
    b->pixel_lds = pl;
    // the single-launch tick: as many workgroups as there are items, at most
    // what the device holds at once, a multiple of the XCD count
    b->tick_lds = std::max(fl, gl);
    int cap = 0;
    KPD_HIP(kpd::tick_capacity(b->tick_lds, &cap));
    const int want = std::max(std::max(b->frame_blocks, b->cell_blocks), (int)b->streams.size());
    b->tick_grid = std::min(cap, (want + 7) / 8 * 8) / 8 * 8;
    drop_graphs(b);
    b->maps_dirty = false;
    return KPD_OK;
}

// Enqueue one tick reading table k: upload, tile pass, mark pass, detection
// of the marked cells, compaction of every stream's D_n (or the one launch
// that does all four); then, when streams may run a per-pixel mask, their
// cell pass, and when a stream asks for them, the features.
hipError_t enqueue_tick(kpd_batch* b, int k)
{
    const size_t n = b->streams.size();
    hipError_t e = hipMemcpyAsync(b->dev_table[k], b->host_table[k], n * sizeof(kpd::TickArgs),
                                  hipMemcpyHostToDevice, b->stream);
    if (b->single_launch && b->tick_grid > 0) {
        if (e == hipSuccess)
            e = kpd::launch_tick(b->dev_table[k], b->dev_fmap, b->frame_blocks, b->dev_cmap, b->cell_blocks, (int)n,
                                 b->dev_sync, k, b->tick_grid, b->tick_lds, b->stream);
        if (e == hipSuccess && b->pixel && b->cell_blocks)
            e = kpd::launch_detect_pixel_batch(b->dev_table[k], b->dev_cmap, b->cell_blocks, b->pixel_lds, b->stream);
        if (e == hipSuccess && b->features && b->cell_blocks)
            e = kpd::launch_describe_batch(b->dev_table[k], b->dev_cmap, b->cell_blocks, b->stream);
        return e;
    }
    if (e == hipSuccess && b->frame_blocks)
        e = kpd::launch_frame_batch(b->dev_table[k], b->dev_fmap, b->frame_blocks, b->frame_lds, b->stream);
    if (e == hipSuccess && b->cell_blocks)
        e = kpd::launch_mark_batch(b->dev_table[k], b->dev_cmap, b->cell_blocks, b->dev_work, b->dev_work_count,
                                   b->stream);
    if (e == hipSuccess && b->cell_blocks)
        e = kpd::launch_detect_list_batch_groups(b->dev_table[k], b->dev_cmap, b->cell_blocks, b->dev_work,
                                                 b->dev_work_count, b->detect_glds, b->stream);
    if (e == hipSuccess && n)
        e = kpd::launch_compact_batch(b->dev_table[k], (int)n, b->dev_work_count, b->stream);
    if (e == hipSuccess && b->pixel && b->cell_blocks)
        e = kpd::launch_detect_pixel_batch(b->dev_table[k], b->dev_cmap, b->cell_blocks, b->pixel_lds, b->stream);
    if (e == hipSuccess && b->features && b->cell_blocks)
        e = kpd::launch_describe_batch(b->dev_table[k], b->dev_cmap, b->cell_blocks, b->stream);
    return e;
}

}  // namespace

extern "C" {

size_t batch_bytes(int max_streams, int max_blocks)
{
    if (max_streams < 1 || max_streams > 65535 || max_blocks < 1) return 0;
    size_t t[2], f, c;
    return batch_layout(max_streams, max_blocks, t, &f, &c);
}

int open_batch(int max_streams, int max_blocks, void* dev_scratch, size_t scratch_bytes, void* hip_stream,
               int use_graph, kpd_batch** out)
{
    if (!out) return fail(KPD_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_streams < 1 || max_streams > 65535 || max_blocks < 1) return fail(KPD_EINVAL, "bad batch capacity");
    size_t t[2], f, c, w, y;
    const size_t need = batch_layout(max_streams, max_blocks, t, &f, &c, &w, &y);
    if (!dev_scratch || reinterpret_cast<uintptr_t>(dev_scratch) % kAlign)
        return fail(KPD_EINVAL, "scratch is NULL or not 256-byte aligned");
    if (scratch_bytes < need) return fail(KPD_ENOMEM, "batch scratch too small");
    kpd_batch* b = new (std::nothrow) kpd_batch();
    if (!b) return fail(KPD_ENOMEM, "host allocation failed");
    if (!kpd::handle_add(b)) {
        delete b;
        return fail(KPD_ENOMEM, "host allocation failed");
    }
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->max_streams = max_streams;
    b->max_blocks = max_blocks;
    b->use_graph = use_graph != 0;
    b->scratch = reinterpret_cast<uint8_t*>(dev_scratch);
    for (int k = 0; k < 2; ++k) b->dev_table[k] = reinterpret_cast<kpd::TickArgs*>(b->scratch + t[k]);
    b->dev_fmap = reinterpret_cast<uint16_t*>(b->scratch + f);
    b->dev_cmap = reinterpret_cast<uint16_t*>(b->scratch + c);
    b->dev_work_count = reinterpret_cast<uint32_t*>(b->scratch + w);
    b->dev_work = reinterpret_cast<uint32_t*>(b->scratch + w + 256);
    b->dev_sync = reinterpret_cast<kpd::TickSync*>(b->scratch + y);
    hipError_t e = hipMemsetAsync(b->dev_work_count, 0, 4, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->dev_sync, 0, sizeof(kpd::TickSync), b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        e = hipHostMalloc(reinterpret_cast<void**>(&b->host_table[k]), (size_t)max_streams * sizeof(kpd::TickArgs),
                          hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->table_free[k], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        close_batch(b);
        return hip_fail(e, "open_batch");
    }
    *out = b;
    return KPD_OK;
}

int batch_set_single_launch(kpd_batch* b, int on)
{
    if (!kpd::handle_live(b)) return fail(KPD_ESTATE, "batch is closed");
    if (on != 0 && on != 1) return fail(KPD_EINVAL, "on must be 0 or 1");
    KPD_HIP(hipStreamSynchronize(b->stream));   // no tick in flight uses the old form
    b->single_launch = on != 0;
    drop_graphs(b);
    return KPD_OK;
}

int batch_attach(kpd_batch* b, kpd_stream* s)
{
    if (!kpd::handle_live(b) || !kpd::handle_live(s)) return fail(KPD_ESTATE, "batch or stream is closed");
    if (s->stream != b->stream) return fail(KPD_EINVAL, "stream was opened on another HIP stream");
    if (s->batch) return fail(KPD_EINVAL, "stream already attached");
    if ((int)b->streams.size() >= b->max_streams) return fail(KPD_ENOMEM, "batch stream capacity exceeded");
    b->streams.push_back(s);
    b->staged.push_back(kpd::TickArgs{});
    b->has_frame.push_back(0);
    const int rc = rebuild_maps(b);
    if (rc != KPD_OK) {
        b->streams.pop_back();
        b->staged.pop_back();
        b->has_frame.pop_back();
        rebuild_maps(b);
    } else {
        s->batch = b;
    }
    return rc;
}

int batch_detach(kpd_batch* b, kpd_stream* s)
{
    if (!kpd::handle_live(b)) return fail(KPD_ESTATE, "batch is closed");
    auto it = std::find(b->streams.begin(), b->streams.end(), s);
    if (it == b->streams.end()) return fail(KPD_EINVAL, "stream not attached");
    const size_t i = (size_t)(it - b->streams.begin());
    if (b->has_frame[i]) return fail(KPD_ESTATE, "stream has a staged frame; tick first");
    b->streams.erase(it);
    b->staged.erase(b->staged.begin() + (long)i);
    b->has_frame.erase(b->has_frame.begin() + (long)i);
    s->batch = nullptr;
    return rebuild_maps(b);
}

}  // extern "C"

namespace {

// Stage stream s's frame; `hint` is where s is first looked for among the
// attached streams (callers pushing in attach order find it there).
int batch_stage(kpd_batch* b, kpd_stream* s, const uint8_t* frame, size_t pitch_bytes, int flags, size_t* hint)
{
    size_t i = *hint;
    if (i >= b->streams.size() || b->streams[i] != s) {
        auto it = std::find(b->streams.begin(), b->streams.end(), s);
        if (it == b->streams.end()) return fail(KPD_EINVAL, "stream not attached");
        i = (size_t)(it - b->streams.begin());
    }
    *hint = i + 1;
    if (b->has_frame[i]) return fail(KPD_ESTATE, "a frame is already staged for this tick");
    const int rc = stage_frame(s, frame, pitch_bytes, flags, &b->staged[i]);
    if (rc != KPD_OK) return rc;
    b->has_frame[i] = 1;
    return KPD_OK;
}

}  // namespace

extern "C" {

int batch_push(kpd_batch* b, kpd_stream* s, const uint8_t* frame, size_t pitch_bytes, int flags)
{
    if (!kpd::handle_live(b)) return fail(KPD_ESTATE, "batch is closed");
    size_t hint = 0;
    return batch_stage(b, s, frame, pitch_bytes, flags, &hint);
}

int batch_push_many(kpd_batch* b, int n, kpd_stream* const* streams, const uint8_t* const* frames,
                    const size_t* pitch_bytes, int flags)
{
    if (!kpd::handle_live(b)) return fail(KPD_ESTATE, "batch is closed");
    if (n < 0 || (n > 0 && (!streams || !frames || !pitch_bytes))) return fail(KPD_EINVAL, "bad arrays");
    size_t hint = 0;
    for (int k = 0; k < n; ++k) {
        const int rc = batch_stage(b, streams[k], frames[k], pitch_bytes[k], flags, &hint);
        if (rc != KPD_OK) return rc;
    }
    return KPD_OK;
}

int batch_tick(kpd_batch* b)
{
    const kpd::TraceRange trace_range("kpd:batch_tick");
    if (!kpd::handle_live(b)) return fail(KPD_ESTATE, "batch is closed");
    if (b->maps_dirty) {
        const int rc = rebuild_maps(b);
        if (rc != KPD_OK) return rc;
    }
    const int k = (int)(b->ticks & 1);
    // the previous upload from this host table must have left it
    if (b->table_used[k]) KPD_HIP(hipEventSynchronize(b->table_free[k]));
    int fbase = 0, cbase = 0;
    bool any = false;
    for (size_t i = 0; i < b->streams.size(); ++i) {
        kpd::TickArgs t = b->has_frame[i] ? b->staged[i] : kpd::TickArgs{};
        const Layout& L = b->streams[i]->L;
        t.active = b->has_frame[i] ? 1 : 0;
        t.tile_base = fbase;
        t.cell_base = cbase;
        fbase += L.tiles_x * L.tiles_y;
        cbase += L.ncell;
        b->host_table[k][i] = t;
        any = any || t.active;
    }
    if (!any) return KPD_OK;
    if (b->use_graph) {
        if (!b->graph[k]) {
            hipGraph_t g = nullptr;
            KPD_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            const hipError_t ce = enqueue_tick(b, k);
            const hipError_t ee = hipStreamEndCapture(b->stream, &g);
            if (ce != hipSuccess) { if (g) (void)hipGraphDestroy(g); return hip_fail(ce, "batch tick capture"); }
            if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
            const hipError_t ie = hipGraphInstantiate(&b->graph[k], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) { b->graph[k] = nullptr; return hip_fail(ie, "hipGraphInstantiate"); }
        }
        KPD_HIP(hipGraphLaunch(b->graph[k], b->stream));
    } else {
        KPD_HIP(enqueue_tick(b, k));
    }
    KPD_HIP(hipEventRecord(b->table_free[k], b->stream));
    b->table_used[k] = true;
    for (size_t i = 0; i < b->streams.size(); ++i)
        if (b->has_frame[i]) {
            advance_frame(b->streams[i], b->staged[i]);
            b->has_frame[i] = 0;
        }
    b->ticks += 1;
    return KPD_OK;
}

int batch_gather(kpd_batch* b, kpd_keypoint* out, size_t out_cap, uint32_t* counts)
{
    if (!kpd::handle_live(b)) return fail(KPD_ESTATE, "batch is closed");
    if (!out || !counts) return fail(KPD_EINVAL, "NULL output");
    if (b->ticks == 0) return fail(KPD_ESTATE, "no tick yet");
    if (b->streams.empty()) return KPD_OK;
    const int k = (int)((b->ticks - 1) & 1);
    const uint32_t cap = out_cap > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)out_cap;
    KPD_HIP(kpd::launch_gather_batch(b->dev_table[k], (int)b->streams.size(), out, cap, counts, b->stream));
    return KPD_OK;
}

int close_batch(kpd_batch* b)
{
    if (!kpd::handle_live(b)) return fail(KPD_ESTATE, "batch is closed");
    const hipError_t e = hipStreamSynchronize(b->stream);
    drop_graphs(b);
    for (int k = 0; k < 2; ++k) {
        if (b->host_table[k]) (void)hipHostFree(b->host_table[k]);
        if (b->table_free[k]) (void)hipEventDestroy(b->table_free[k]);
    }
    for (kpd_stream* s : b->streams) s->batch = nullptr;   // they stay open, detached
    kpd::handle_remove(b);
    delete b;
    if (e != hipSuccess) return hip_fail(e, "close_batch");
    return KPD_OK;
}

int kpd_pyramid_level(kpd_stream* s, int octave, uint8_t* out)
{
    if (!kpd::handle_live(s)) return fail(KPD_ESTATE, "stream is closed");
    if (s->n_pushed == 0) return fail(KPD_ESTATE, "no frame pushed yet");
    if (octave < 1 || octave >= s->L.O || !out) return fail(KPD_EINVAL, "bad octave or NULL output");
    const Layout& L = s->L;
    const size_t copy = s->chunk_n > 0 ? (size_t)(s->chunk_n - 1) : 0;   // the last frame's octaves
    const uint8_t* src = s->arena + L.pyr_stride * copy + L.off_lvl[octave];
    if (alternates(s, octave) && s->layer_buf == 1) src = alt_level(s, octave);
    KPD_HIP(hipMemcpy2DAsync(out, L.w[octave], src, L.pitch[octave], L.w[octave], L.h[octave], hipMemcpyDeviceToHost,
                             s->stream));
    KPD_HIP(hipStreamSynchronize(s->stream));
    return KPD_OK;
}

}  // extern "C"
