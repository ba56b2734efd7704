/*
 * kpd.h — C ABI of the MI355X (gfx950) masked multi-scale keypoint detector
 * for video.
 *
 * The library implements the detection path of Baroffio et al., "Fast
 * keypoint detection in video sequences" (arXiv:1503.06959):
 *   - each frame I_n (Sec. 3) is split into an N_r x N_c grid of cells, the
 *     bins of Sec. 3.2;
 *   - a cell is marked for detection when its mean absolute frame-to-frame
 *     difference exceeds T_I (Sec. 3.1, Eq. 2, with the polarity the text
 *     describes: detect where the frame changes) or when the previous frame
 *     left at least T_H keypoints in it (Sec. 3.2, Eqs. 3-4); the two tests
 *     are OR-ed;
 *   - in marked cells the FAST-9/16 segment test (Sec. 2, AST on the radius-3
 *     Bresenham circle, threshold t) runs on every octave of a 2x2-box
 *     pyramid (Sec. 2, Sec. 3.1), scores candidates with the FAST score
 *     V = max(sum of (c - p - t) over brighter ring pixels, sum of
 *     (p - c - t) over darker ones), and keeps the maxima of a 3x3
 *     scale-space neighbourhood (Sec. 2);
 *   - unmarked cells carry their previous keypoints forward (Sec. 3, Eq. 1).
 *
 * Memory and streams. The caller owns all device memory: it allocates one
 * device arena per stream of at least stream_bytes() bytes (e.g. a torch
 * uint8 tensor) and keeps it alive until close_stream(). The library never
 * allocates or frees device memory. Work is enqueued on the caller's HIP
 * stream (hipStream_t passed as void*; NULL = the default stream).
 * Processes that also use PyTorch must load PyTorch first, so that both use
 * one HIP runtime.
 *
 * Errors. Every call returns 0 (KPD_OK) or a negative KPD_E* code; a
 * thread-local message is available from kpd_last_error(). No C++ exception
 * crosses the ABI. One handle must not be used from two threads at once.
 */
#ifndef KPD_H
#define KPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KPD_OK 0
#define KPD_EINVAL (-1)   /* bad parameters, sizes, pitch or flags */
#define KPD_ENOMEM (-2)   /* arena smaller than stream_bytes() */
#define KPD_EDEVICE (-3)  /* a HIP call failed; see kpd_last_error() */
#define KPD_ETRUNC (-4)   /* output capacity too small; *count holds the need */
#define KPD_ESTATE (-5)   /* call out of order (get before push, closed handle) */

#define KPD_KB_OFF 0xFFFFFFFFu  /* kb_thresh value that switches binning off */
#define KPD_MAX_OCTAVES 8
#define KPD_MAX_CELL 128        /* largest cell side, in level-0 pixels */
#define KPD_MAX_DIM 16384       /* largest frame side */
#define KPD_MAX_CHUNK 512       /* most frames per push_frames call */

/* push_frame flags */
#define KPD_FRAME_HOST 0          /* host pointer; copied into the arena */
#define KPD_FRAME_DEVICE 1        /* device pointer; copied into the arena */
#define KPD_FRAME_DEVICE_RETAIN 2 /* device pointer used in place (no copy) */

/* Detector and mask parameters.
 *   fast_t     AST threshold t (Sec. 2), 1..254.
 *   n_octaves  number of pyramid levels O, counting level 0; 1..KPD_MAX_OCTAVES,
 *              with (width >> (O-1)) >= 1 and (height >> (O-1)) >= 1.
 *   grid_cols, grid_rows
 *              N_c x N_r cell grid (Sec. 3.2). Level-0 pixel (X,Y) lies in
 *              cell (floor(X*N_c/W), floor(Y*N_r/H)); every cell side must be
 *              at most KPD_MAX_CELL pixels.
 *   id_thresh  T_I: a cell is marked when its summed |I_n - I_{n-1}| exceeds
 *              T_I times its pixel count. Negative: every cell is marked
 *              (full-frame detection); >= 255: the test never fires.
 *   kb_thresh  T_H: a cell is marked when D_{n-1} has >= T_H keypoints in it
 *              (Eq. 4). 0: every cell is marked; KPD_KB_OFF: never fires.
 *   tile       side of the level-0 tiles of the pyramid/difference pass of
 *              single-frame pushes and batch ticks, a tuning knob that
 *              never changes results: 0 picks the default (the widest of
 *              128, 64, 32 that gives the frame at least 128 tiles, at
 *              least 2^(O-1)), otherwise a power of two in 32..128 and
 *              >= 2^(O-1). Chunks (push_frames) use their own tiles.
 *   chunk_frames
 *              most frames one push_frames call may take (0 or 1: the
 *              stream takes single frames only; at most KPD_MAX_CHUNK). It
 *              sizes the arena.
 *   layer_mask 1: the stream may switch to the per-pixel masks
 *              (set_mask_mode); a second copy of octaves 1..O-1 keeps the
 *              previous frame's readable. Eq. 1 per feature can then place a carried
 *              and a new feature side by side, so D_n is sized for every
 *              decision pixel instead of one feature per 2x2 block. 0: no.
 *   features   what every feature of D_n carries besides its keypoint,
 *              computed for the keypoints new in D_n and carried with the
 *              others (Sec. 3, Eq. 1): KPD_FEAT_DESCRIPTOR, an orientation
 *              sector and a 512-bit binary descriptor (get_descriptors);
 *              KPD_FEAT_REFINE, the sub-pixel position and sub-scale of
 *              Sec. 2's interpolation (get_refined). push_frame,
 *              push_frames (get_chunk_descriptors, get_chunk_refined) and
 *              batch ticks, in every mask mode (with a per-pixel mask,
 *              set_mask_mode 1 or 2, a marked cell holds new and carried
 *              features side by side). 0: nothing.
 *   group_cols, group_rows
 *              cells one detection workgroup covers when a chunk's
 *              parameters mark every cell (full-frame detection): a
 *              rectangle of group_cols x group_rows cells shares one pixel
 *              tile and one score map per octave. A tuning knob that never
 *              changes results: 0, 0 picks the default; otherwise
 *              1..grid_cols and 1..grid_rows.
 *   group_threads
 *              threads of those workgroups: 0 (the default, 256), 256 or
 *              512; never changes results. */
typedef struct kpd_params {
    int32_t fast_t;
    int32_t n_octaves;
    int32_t grid_cols;
    int32_t grid_rows;
    int32_t id_thresh;
    uint32_t kb_thresh;
    int32_t tile;
    int32_t chunk_frames;
    int32_t layer_mask;
    int32_t features;
    int32_t group_cols;
    int32_t group_rows;
    int32_t group_threads;
} kpd_params;

#define KPD_FEAT_DESCRIPTOR 1
#define KPD_FEAT_REFINE 2

/* One feature of D_n (Sec. 3: position and scale; the integer part).
 * x, y are coordinates at level `octave`; the level-0 footprint starts at
 * (x << octave, y << octave), and that point decides the keypoint's cell.
 * score is the FAST score V (9..4064). */
typedef struct kpd_keypoint {
    uint16_t x;
    uint16_t y;
    uint8_t octave;
    uint8_t pad;
    uint16_t score;
} kpd_keypoint;

typedef struct kpd_stream kpd_stream;

/* Device arena bytes a stream of this shape needs; 0 when the parameters are
 * invalid. Pure host computation. */
size_t stream_bytes(int width, int height, const kpd_params* params);

/* Open a video stream (Sec. 3: the sequence I_0, I_1, ...). `dev_arena` is a
 * device pointer to `arena_bytes` bytes owned by the caller, 256-byte
 * aligned. `hip_stream` is the hipStream_t all work goes to. O and the grid
 * are fixed for the stream's life. The library allocates no device memory;
 * it takes a small pinned host buffer (under 40 KB plus a byte per cell) for
 * reading results back. Returns KPD_EINVAL for bad parameters, KPD_ENOMEM
 * when arena_bytes < stream_bytes(). */
int open_stream(int width, int height, const kpd_params* params, void* dev_arena,
                size_t arena_bytes, void* hip_stream, kpd_stream** out);

/* Change the AST threshold t (Sec. 2), the intensity-difference threshold
 * T_I (Sec. 3.1, Eq. 2) and the keypoint-count threshold T_H (Sec. 3.2,
 * Eqs. 3-4) from the next pushed frame on. A change of t re-marks every cell
 * of the next frame, since carried scores depend on t. KPD_EINVAL when t is
 * outside 1..254, KPD_ESTATE on a closed handle. */
int set_thresholds(kpd_stream* s, int32_t fast_t, int32_t id_thresh, uint32_t kb_thresh);

/* Process the next frame I_n (Sec. 3: uint8 grey, width x height, rows
 * `pitch_bytes` apart, pitch >= width): the cell mask M_n (Sec. 3.1 Eq. 2
 * read per cell, Sec. 3.2 Eqs. 3-4), the octave pyramid and detection in
 * the marked cells (Sec. 2), and D_n by Eq. 1 (new keypoints of marked
 * cells, D_{n-1}'s of the others). Asynchronous: enqueues the kernels and
 * returns; KPD_EINVAL for a bad pitch or flag, KPD_EDEVICE when a launch
 * fails. Flags:
 *   KPD_FRAME_HOST           `frame` is host memory, copied into the arena;
 *                            it must stay valid until the stream has
 *                            synchronised (get_keypoints does).
 *   KPD_FRAME_DEVICE         `frame` is device memory, copied into the arena.
 *   KPD_FRAME_DEVICE_RETAIN  `frame` is device memory read in place; it must
 *                            stay valid and unchanged until the work of the
 *                            NEXT push_frame has completed (it is I_{n-1}
 *                            then). */
int push_frame(kpd_stream* s, const uint8_t* frame, size_t pitch_bytes, int flags);

/* Process `n_frames` consecutive frames (1 <= n_frames <= chunk_frames) in
 * one pass of three to six launches: a pyramid/difference pass over all of
 * them, the mark passes (none when the parameters mark every cell), a
 * detection pass over the marked (frame, cell) items or, when every cell is
 * marked, over every (frame, group of cells), and a compaction pass per
 * frame that applies Eq. 1.
 * Frame i is the device buffer frames + i * frame_stride (rows pitch_bytes
 * apart), read in place under the KPD_FRAME_DEVICE_RETAIN rules (the last
 * frame is I_{n-1} of the next push). Results are exactly those of pushing
 * the frames one by one: get_keypoints then returns the last frame's D_n,
 * and kpd_chunk_result every frame's. KPD_EINVAL if the stream was opened
 * without chunk_frames >= 2. */
int push_frames(kpd_stream* s, const uint8_t* frames, size_t frame_stride, size_t pitch_bytes, int n_frames);

/* Mask mode from the next push_frame on (a change re-detects every cell of
 * that frame). mode 0: the per-cell test of Sec. 3.1 Eq. 2 read as a mean
 * absolute level-0 difference per cell (the default). mode 1: Eq. 2 per
 * pixel of pyramid layer `layer` (0..n_octaves-1; the paper uses the top
 * layer), one mask for all octaves, replicated to level 0 (level-0 pixel
 * (X,Y) takes layer pixel (X >> layer, Y >> layer), clamped to the layer's
 * last column and row), and Eq. 1 applied per feature at its level-0
 * position (x << octave, y << octave); T_H still marks whole cells. mode 2
 * (layer must be 0): Sec. 3.1's one mask per octave, Eq. 2 per pixel of
 * every level, a feature at level o tested on level o's pixel (x, y). The
 * reported cell mask flags cells marked by T_H or holding a changed pixel
 * (of any level, replicated to level 0, in mode 2). Modes 1 and 2 run on
 * push_frame, in batch ticks (whose batch then adds one launch per tick
 * for the cells of its streams opened with layer_mask) and on push_frames
 * (there with T_H off, KPD_KB_OFF, unless every cell is marked anyway: a
 * chunk's per-pixel marks cannot depend on the counts of the frame before).
 * Either mode returns KPD_EINVAL on a stream opened without layer_mask. */
int set_mask_mode(kpd_stream* s, int mode, int layer);

/* Orientation and binary descriptor of one feature (Sec. 3: a feature is
 * position, scale, orientation and a binary descriptor). The pattern is 60
 * points in pixels of the keypoint's level: the centre and rings of
 * (radius, points) (3, 10), (5, 14), (7.5, 15), (11, 20), point i of a ring
 * of n at angle 2*pi*i/n, offsets rounded half away from zero, each point
 * the mean of a box of half-size 1 (centre, inner two rings) or 2 (outer
 * rings), edge pixels repeated outside the level. `sector` (0..31) is the
 * angle of the sum over point pairs at squared distance >= 169 of
 * (p_j - p_i)(V_j - V_i), in 32 equal sectors; `bits` holds, for the 512
 * shortest pairs (squared distance < 96, by distance then indices), bit k
 * = V_a > V_b with the pattern turned by 2*pi*sector/32 (bit k in word
 * k / 64, bit k % 64). */
typedef struct kpd_descriptor {
    uint32_t sector;
    uint32_t pad;
    uint64_t bits[8];
} kpd_descriptor;

/* Descriptors of D_n, in get_keypoints' order (streams opened with
 * KPD_FEAT_DESCRIPTOR). `*count` receives the number of features; when it
 * exceeds `capacity`, nothing is copied and KPD_ETRUNC is returned.
 * KPD_EINVAL without descriptors, KPD_ESTATE before the first push. */
int get_descriptors(kpd_stream* s, kpd_descriptor* out, size_t capacity, size_t* count);

/* The descriptor pattern's point i (0..59) turned to `sector` (0..31):
 * rounded offsets in level pixels and the box half-size (returned; -1 for
 * out-of-range arguments). Host only, no stream needed. */
int kpd_desc_point(int sector, int i, int* dx, int* dy);

/* Sub-pixel position and sub-scale of one feature (Sec. 2's interpolation,
 * on the octave layers). On the keypoint's layer and the finer and coarser
 * ones (centres (x, y), (2x+1, 2y+1), (x>>1, y>>1)), a least-squares
 * quadratic through the 3 x 3 FAST scores (0 outside the candidate region)
 * gives a maximum, clamped to one pixel and taken at the centre when the fit
 * is not concave; a parabola through the three maxima along log2 scale gives
 * t in [-1, 1] (0 when not concave; a missing layer counts 0); x, y (level-0
 * pixels, pixel (X, Y) spanning [X, X+1) x [Y, Y+1)) move from the own
 * layer's maximum towards the coarser (t > 0) or finer (t < 0) one's by |t|;
 * log2_scale = octave + t; score = the parabola's value at t. Every
 * floating step is an IEEE double operation in a fixed order, then rounded
 * to float. */
typedef struct kpd_refined {
    float x;
    float y;
    float log2_scale;
    float score;
} kpd_refined;

/* Refined values of D_n, in get_keypoints' order (streams opened with
 * KPD_FEAT_REFINE); like get_descriptors otherwise. */
int get_refined(kpd_stream* s, kpd_refined* out, size_t capacity, size_t* count);

/* Wait for the last pushed frame and copy D_n (Sec. 3's feature set of
 * frame n, Eq. 1) to host memory `out`, ordered by cell (row-major), then
 * octave, then y, then x. `*count` receives the
 * number of keypoints; when it exceeds `capacity`, nothing is copied and
 * KPD_ETRUNC is returned. `cell_mask` (nullable, N_r*N_c bytes, row-major)
 * receives M_n (1 = detected this frame, 0 = carried). KPD_ESTATE before the
 * first push. */
int get_keypoints(kpd_stream* s, kpd_keypoint* out, size_t capacity, size_t* count,
                  uint8_t* cell_mask);

/* Release the handle (waits for its queued work). The arena may be freed
 * afterwards. A stream attached to a batch is detached first (KPD_ESTATE,
 * and the stream stays open, when it has a frame staged for the next tick).
 * Every later call with the handle, close_stream included, returns
 * KPD_ESTATE: the library keeps a set of the handles it has handed out and
 * not released, and checks each handle against it (until a new handle
 * happens to reuse the address). */
int close_stream(kpd_stream* s);

/* Forget the previous frame (e.g. at a scene cut): the next pushed frame is
 * treated like the first frame of a stream, which has no I_{n-1} or D_{n-1}
 * to build a mask from, and re-detects every cell. Does not synchronise. */
int reset_stream(kpd_stream* s);

/* Message of the last failing call on this thread ("" when none). */
const char* kpd_last_error(void);

/* ------------------------------------------------------------- batching */

/* A batch runs the next frame of many streams (of any sizes and parameters)
 * in one tick, optionally replayed from a captured HIP graph. By default a
 * tick is four launches (tile passes; marks with the marked cells listed;
 * detection of the listed cells; each stream's D_n by Eq. 1);
 * batch_set_single_launch(b, 1) makes it one launch of co-resident
 * workgroups whose phases are separated by device-wide barriers. When an
 * attached stream was opened with layer_mask, one more launch runs the
 * cells of the streams with a per-pixel mask set (set_mask_mode); when an
 * attached stream computes features (descriptors or refined values), one
 * more launch computes them for every such stream. Results are exactly
 * those of pushing each stream's frame alone. */
typedef struct kpd_batch kpd_batch;

/* Device scratch bytes of a batch holding up to `max_streams` streams whose
 * tiles and cells need at most `max_blocks` workgroups per launch. */
size_t batch_bytes(int max_streams, int max_blocks);

/* Open a batch on `hip_stream`; `dev_scratch` (caller-owned, 256-byte
 * aligned, >= batch_bytes()) holds the tick tables. use_graph = 1 captures
 * each tick's table upload and launches once per set of attached streams
 * and replays it. */
int open_batch(int max_streams, int max_blocks, void* dev_scratch, size_t scratch_bytes, void* hip_stream,
               int use_graph, kpd_batch** out);

/* Attach or detach a stream. The stream must have been opened on the
 * batch's HIP stream and may belong to one batch at a time (KPD_EINVAL
 * otherwise). KPD_ENOMEM when the batch's stream or workgroup capacity
 * would be exceeded. */
int batch_attach(kpd_batch* b, kpd_stream* s);
int batch_detach(kpd_batch* b, kpd_stream* s);

/* Stage the next frame of an attached stream for the next tick (same frame
 * and flag rules as push_frame; a copy is enqueued at once). At most one
 * frame per stream per tick: KPD_ESTATE if one is already staged. */
int batch_push(kpd_batch* b, kpd_stream* s, const uint8_t* frame, size_t pitch_bytes, int flags);

/* Stage the next frame of n attached streams in one call: the same as n
 * batch_push calls in array order (streams[k] gets frames[k] with row pitch
 * pitch_bytes[k], all with `flags`), for servers that stage hundreds of
 * streams per tick. Stops at the first failure and returns its code; the
 * frames before it stay staged. */
int batch_push_many(kpd_batch* b, int n, kpd_stream* const* streams, const uint8_t* const* frames,
                    const size_t* pitch_bytes, int flags);

/* Run one tick over every attached stream with a staged frame.
 * Asynchronous; get_keypoints on a stream waits for it. A barrier wait of
 * the single-launch tick that does not end (the device holding fewer of its
 * workgroups than it was sized for) gives up after about a second and makes
 * get_keypoints of the ticked streams return KPD_EDEVICE. */
int batch_tick(kpd_batch* b);

/* Tick form: 1 one launch per tick, 0 (the default) four launches. Waits
 * for the batch's queued work; results do not depend on the form. */
int batch_set_single_launch(kpd_batch* b, int on);

/* Gather the results of the last tick: counts[i] (uint32, device memory)
 * receives the size of D_n of the i-th attached stream (attach order; 0 for
 * streams without a frame in that tick), and `out` (device memory, `out_cap`
 * entries) their keypoints concatenated in that order, each stream's in
 * D_n's own order. Entries past out_cap are dropped; the counts still report
 * full sizes. Asynchronous on the batch's HIP stream; must follow the tick
 * it gathers, before the next tick. */
int batch_gather(kpd_batch* b, kpd_keypoint* out, size_t out_cap, uint32_t* counts);

/* Wait for the batch's work and release it. Attached streams stay open,
 * detached. */
int close_batch(kpd_batch* b);

/* ------------------------------------------------------- inspection calls */

/* Device-resident result of the last frame: pointer to the D_n list and to
 * its uint32 length, valid until the next push_frame. Does not synchronise. */
int kpd_device_result(kpd_stream* s, const kpd_keypoint** d_list, const uint32_t** d_count);

/* Device-resident D_n of frame i (0-based) of the last push_frames call:
 * pointer to the list and to its uint32 length, valid until the next push.
 * Does not synchronise. */
int kpd_chunk_result(kpd_stream* s, int i, const kpd_keypoint** d_list, const uint32_t** d_count);

/* Wait and copy D_n of frame i (0-based) of the last push_frames call to
 * host memory, with get_keypoints' count/capacity rules (KPD_ETRUNC with
 * *count set when capacity is too small). */
int get_chunk_keypoints(kpd_stream* s, int i, kpd_keypoint* out, size_t capacity, size_t* count);

/* Descriptors and refined values (Sec. 3 feature model, Sec. 2's
 * interpolation; Eq. 1 carries them with their keypoints) of frame i of the
 * last push_frames call, in get_chunk_keypoints' order: a feature is
 * described on the levels of the frame that detected it. Streams opened
 * with KPD_FEAT_DESCRIPTOR / KPD_FEAT_REFINE (KPD_EINVAL otherwise);
 * count/capacity rules as get_chunk_keypoints'. */
int get_chunk_descriptors(kpd_stream* s, int i, kpd_descriptor* out, size_t capacity, size_t* count);
int get_chunk_refined(kpd_stream* s, int i, kpd_refined* out, size_t capacity, size_t* count);

/* Wait and copy per-cell statistics of the last frame: the summed absolute
 * level-0 difference (uint32 per cell; meaningful only on frames whose mask
 * was computed from data, i.e. not the first frame, not after a change of t,
 * and not with T_I < 0 or T_H == 0) and the per-cell keypoint count of D_n.
 * Either pointer may be NULL. */
int kpd_cell_stats(kpd_stream* s, uint32_t* sad, uint32_t* counts);

/* Wait and copy pyramid level o (1 <= o < O) of the last frame into `out`
 * ((width >> o) x (height >> o) bytes, row-major, no padding). */
int kpd_pyramid_level(kpd_stream* s, int octave, uint8_t* out);

/* ------------------------------------------------------ kernel timing */

/* Kernels of one push, in launch order: the pyramid-and-SAD pass over
 * level-0 tiles, the per-cell detection pass, and (push_frames only) the
 * compaction pass that builds each frame's D_n in cell order. */
#define KPD_K_FRAME 0
#define KPD_K_DETECT 1
#define KPD_K_COMPACT 2 /* compaction pass (Eq. 1) of push_frame and push_frames */
#define KPD_K_MARK 3    /* mark, speculation and resolve passes of push_frames */
#define KPD_K_DESCRIBE 4 /* feature pass of push_frame and push_frames: descriptors, refinement */
#define KPD_NKERNELS 5

/* Switch per-kernel GPU timing on (1) or off (0). While on, every kernel
 * launch of this stream is bracketed by two HIP events recorded on the
 * stream's HIP stream; the library creates the events on first use and keeps
 * them until close_stream. */
int kpd_profile(kpd_stream* s, int enable);

/* Wait for the stream, then add up the event-timed durations since the last
 * read: ms[k] receives the summed milliseconds of kernel k and launches[k]
 * the number of launches (arrays of KPD_NKERNELS; either may be NULL). */
int kpd_profile_read(kpd_stream* s, double* ms, uint64_t* launches);

/* ------------------------------------------ octaves and intra-octaves */

/* Full-frame detection of one frame over BRISK's scale space with the
 * layers between the octaves (Sec. 2). Layers in scale order c_0, d_0,
 * c_1, d_1, ..., c_{O-1}, d_{O-1} (layer index 2i for c_i, 2i+1 for d_i):
 * c_i are the octaves of push_frame (2x2 means, round half up, sizes
 * halved by floor); d_0 takes every whole 3x3 block of the frame to a 2x2
 * block, output (2a+p, 2b+q) = (sum of w_p(i) w_q(j) I(3a+i, 3b+j) + 4) / 9
 * with w_0 = (2,1,0), w_1 = (0,1,2) (the rounded mean over the 1.5 x 1.5
 * area it covers; size floor(W/3)*2 x floor(H/3)*2); d_{i+1} halves d_i.
 * A pixel of c_i spans 2^i level-0 pixels a side, one of d_i 1.5 * 2^i.
 * Every layer is scored like the octaves (FAST-9/16 score, no candidates
 * within 3 pixels of a layer's border). Two pixels of one layer, or of
 * layers adjacent in the scale order, are neighbours when their closed
 * level-0 footprints [x s, (x+1) s] x [y s, (y+1) s] intersect; between
 * two octaves this is push_frame's neighbourhood. A pixel with score > 0 is
 * a keypoint when no neighbour ranks above it (higher score, then the lower
 * layer, then the smaller (y, x)).
 *
 * frame: device, `pitch_bytes` per row; workspace: device, 256-byte
 * aligned, at least kpd_layers_bytes() bytes, used by one call at a time;
 * out: device, `capacity` kpd_keypoint records in (layer, y, x) order, the
 * `octave` field holding the layer index (entries past capacity are
 * dropped); count: device uint32 receiving the keypoint total. All work is
 * queued on `hip_stream`; nothing is read back. */
size_t kpd_layers_bytes(int width, int height, int n_octaves);
int kpd_detect_layers(const uint8_t* frame, size_t pitch_bytes, int width, int height, int fast_t, int n_octaves,
                      void* workspace, size_t workspace_bytes, kpd_keypoint* out, uint32_t capacity, uint32_t* count,
                      void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * kpd_detect_layers with its workspace in a static device array of
 * KPD_STATIC_WORKSPACE bytes, which the library keeps on every GPU it runs
 * on until the process ends. Frames whose kpd_layers_bytes() exceeds it
 * (1920 x 1080 fits) return KPD_EINVAL. Every call on one GPU shares the
 * array, which keeps the last call's layers and score maps: calls that
 * overlap on one GPU race, so queue them on one HIP stream. `hip_stream`
 * must belong to the current device. Other arguments, ownership and errors
 * as kpd_detect_layers; allocates nothing. */
#define KPD_STATIC_WORKSPACE (16u << 20)
int kpd_detect_layers_static(const uint8_t* frame, size_t pitch_bytes, int width, int height, int fast_t,
                             int n_octaves, kpd_keypoint* out, uint32_t capacity, uint32_t* count, void* hip_stream);

/* Refinement of keypoints on these layers (Sec. 2's sub-pixel and
 * sub-scale interpolation over the layered scale space), from the score
 * maps that the last kpd_detect_layers call left in `workspace`. For a
 * keypoint (x, y) of layer l, layers l-1, l, l+1 are fitted as
 * get_refined's layers are (3 x 3 scores, exact integer least squares,
 * maximum clamped to a pixel) at the pixel holding the keypoint's footprint
 * centre, floor((2x+1) S_l / (2 S_m)) with S the pixel size in half
 * level-0 pixels. Layer m sits at log2 scale sigma_m = m/2 for octaves and
 * (m-1)/2 + log2(1.5) for intra-octaves (log2(1.5) rounded to double; a
 * missing layer below c_0 or past the last has value 0 and the keypoint's
 * position). The parabola through the three values in Newton form, d1 =
 * (m_1 - m_0)/(sigma_1 - sigma_0), d2 = (m_2 - m_1)/(sigma_2 - sigma_1),
 * c = (d2 - d1)/(sigma_2 - sigma_0), has its vertex at (sigma_0 + sigma_1)/2
 * - d1/(2c) when c < 0 (clamped to [sigma_0, sigma_2]), else sigma_1; the
 * score is its value there, log2_scale the vertex, and x, y move from the
 * own layer's maximum towards the coarser (vertex above sigma_1) or finer
 * one's by the fraction of the way in log2 scale. IEEE double steps in a
 * fixed order, rounded to float.
 * list, count: device keypoints of the last detection and their device
 * count (the out/count given to it); out: device, min(count, capacity)
 * records written in list order. */
int kpd_refine_layers(int width, int height, int n_octaves, void* workspace, size_t workspace_bytes,
                      const kpd_keypoint* list, const uint32_t* count, uint32_t capacity, kpd_refined* out,
                      void* hip_stream);

/* The masked stream over octaves and intra-octaves: push_frame's per-cell
 * mask (the level-0 difference test against id_thresh, the count test of
 * D_{n-1} against kb_thresh, every cell on the first frame and after
 * kpd_lstream_reset) and Eq. 1, with F(I_n) the detection of
 * kpd_detect_layers. A keypoint (x, y) of layer l lies in the cell of its
 * level-0 footprint start (floor(x S_l / 2), floor(y S_l / 2)), S_l in half
 * pixels (push_frame's rule for the octaves), for the count test, for Eq. 1
 * and for D_n's order: cell, then layer, then y, then x. The `octave` field
 * holds the layer index. Parameters used: fast_t, n_octaves, grid_cols,
 * grid_rows, id_thresh, kb_thresh, chunk_frames. Frames and flags as
 * push_frame. */
typedef struct kpd_lstream kpd_lstream;
size_t kpd_lstream_bytes(int width, int height, const kpd_params* params);
int kpd_lstream_open(int width, int height, const kpd_params* params, void* dev_arena, size_t arena_bytes,
                     void* hip_stream, kpd_lstream** out);
int kpd_lstream_push(kpd_lstream* s, const uint8_t* frame, size_t pitch_bytes, int flags);
/* D_n and, when cell_mask is not NULL, M_n (one byte per cell); like
 * get_keypoints (synchronises; KPD_ETRUNC copying nothing when D_n exceeds
 * capacity). */
int kpd_lstream_get(kpd_lstream* s, kpd_keypoint* out, size_t capacity, size_t* count, uint8_t* cell_mask);
/* n_frames consecutive device frames (1 <= n_frames <= chunk_frames) in one
 * pass of a few launches, read in place as push_frames reads them: the
 * marks of every frame, the layers of every frame, scores and suppression
 * in the cells the marks need, the marked cells' keypoints, and each
 * frame's D by Eq. 1. kb_thresh must be KPD_KB_OFF unless id_thresh < 0 or
 * kb_thresh == 0 mark every cell anyway (KPD_EINVAL): the count test would
 * chain a chunk's marks frame by frame. Results are exactly those of
 * pushing the frames one by one: kpd_lstream_get returns the last frame's
 * D_n and M_n, kpd_lstream_get_chunk frame i's D (count/capacity rules as
 * kpd_lstream_get). */
int kpd_lstream_push_frames(kpd_lstream* s, const uint8_t* frames, size_t frame_stride, size_t pitch_bytes,
                            int n_frames);
int kpd_lstream_get_chunk(kpd_lstream* s, int i, kpd_keypoint* out, size_t capacity, size_t* count);

/* A batch of masked streams over the layers that share one frame size and
 * one set of parameters: max_streams slots, each a stream of its own with
 * kpd_lstream's rules, advanced together by ticks. A tick runs every slot
 * with a staged frame in a fixed set of launches (the marks of every slot's
 * cells, the layers of every slot's frame, scores and suppression where
 * the marks need them, each slot's D_n by Eq. 1); slots without a frame keep
 * their state. Results are exactly those of one kpd_lstream per slot.
 * Parameters used: those of kpd_lstream but chunk_frames. The arena
 * (caller-owned device memory, 256-byte aligned, >= kpd_lbatch_bytes)
 * holds every slot's state. */
typedef struct kpd_lbatch kpd_lbatch;
size_t kpd_lbatch_bytes(int width, int height, const kpd_params* params, int max_streams);
int kpd_lbatch_open(int width, int height, const kpd_params* params, int max_streams, void* dev_arena,
                    size_t arena_bytes, void* hip_stream, kpd_lbatch** out);
/* Stage slot's next frame: device memory read in place, as push_frame's
 * KPD_FRAME_DEVICE_RETAIN frames (it must stay unchanged until the slot's
 * next tick has completed, which reads it as I_{n-1}). KPD_ESTATE when a
 * frame is already staged for the slot. */
int kpd_lbatch_push(kpd_lbatch* b, int slot, const uint8_t* frame, size_t pitch_bytes);
/* Run one tick (asynchronous on the batch's HIP stream). */
int kpd_lbatch_tick(kpd_lbatch* b);
/* Slot's D_n and M_n after its last tick, as kpd_lstream_get (waits);
 * KPD_ESTATE before the slot's first tick. */
int kpd_lbatch_get(kpd_lbatch* b, int slot, kpd_keypoint* out, size_t capacity, size_t* count, uint8_t* cell_mask);
/* The slot's next frame is treated as a first frame. */
int kpd_lbatch_reset(kpd_lbatch* b, int slot);
int kpd_lbatch_close(kpd_lbatch* b);
int kpd_lstream_reset(kpd_lstream* s);
int kpd_lstream_close(kpd_lstream* s);

/* Where layer `layer` (1 .. 2 n_octaves - 1; layer 0 is the frame) lies in
 * the workspace after kpd_detect_layers: byte offset, width and height,
 * rows packed (pitch = width). */
int kpd_layer_plane(int width, int height, int n_octaves, int layer, size_t* offset, int* w, int* h);

/* ------------------------------------------ temporally coherent detector */

/* The comparison system of Sec. 4: keypoints propagated from frame to frame
 * by block matching instead of being detected. Frames come in groups of
 * `gop` (Delta), counted from the first push and from tcd_reset. The first
 * frame of a group takes the full-frame detection F(I_n) (as push_frame with
 * T_I < 0, in D_n's order); every keypoint becomes a track at the centre of
 * its level-0 footprint, 4(x << o) + 2(2^o - 1) in quarter pixels (likewise
 * y). Every other frame moves each track of the previous frame:
 *   - a sample at quarter position (X, Y) = (4x + a, 4y + b) is the exact
 *     bilinear mix ((4-a)(4-b) I(x,y) + a(4-b) I(x+1,y) + (4-a)b I(x,y+1)
 *     + ab I(x+1,y+1) + 8) >> 4;
 *   - a patch is the 16 x 16 samples at (X + 4(i-8), Y + 4(j-8)); a
 *     position is usable when X >= 32, Y >= 32, X + 28 <= 4(W-2) and
 *     Y + 28 <= 4(H-2); a track whose patch in I_{n-1} is not usable is
 *     dropped;
 *   - the coarse step tries displacements of (2u, 2v) pixels, |u|, |v| <= 6
 *     (the 24-pixel window at a precision of 2), the fine step, around the
 *     coarse winner, (u/4, v/4) pixels, |u|, |v| <= 7 (quarter pixels up to
 *     1.75 away). Each step visits its grid in spiral order (ring
 *     max(|u|,|v|) outwards, each ring clockwise from its top-left corner,
 *     y down), skips unusable candidates, keeps the lowest SAD against the
 *     track's patch in I_{n-1} (the earliest on ties) and stops at the first
 *     SAD below t_et;
 *   - the track moves to the fine winner when its SAD is below t_bm, and is
 *     dropped otherwise. Survivors keep their order.
 * Integer arithmetic throughout. The tracker owns an inner stream (tcd_bytes
 * includes it) and two frame slots in its arena. */
typedef struct kpd_tcd_params {
    int32_t gop;    /* frames per group (Delta), >= 1; the paper uses 10 */
    int32_t t_bm;   /* a match needs SAD < t_bm (the paper's T_BM = 1800) */
    int32_t t_et;   /* a step stops at the first SAD < t_et (T_ET = 1000; 0: never) */
    int32_t pad;    /* 0 */
} kpd_tcd_params;

typedef struct kpd_track {
    int32_t x4, y4;   /* position in quarter pixels of level 0 */
    uint8_t octave;   /* of the detection the track started from */
    uint8_t pad;
    uint16_t score;   /* FAST score at detection */
    uint32_t sad;     /* SAD of the last match (0 on the group's first frame) */
} kpd_track;

typedef struct kpd_tcd kpd_tcd;

/* Arena bytes for a tracker on width x height frames. `det` holds the
 * detector's fast_t, n_octaves, grid and tile (its id_thresh, kb_thresh,
 * chunk_frames, layer_mask and features are ignored: the group's first
 * frame is detected whole). 0 when invalid (see kpd_last_error). */
size_t tcd_bytes(int width, int height, const kpd_params* det, const kpd_tcd_params* tp);

/* Open a tracker on a caller-owned, 256-byte-aligned device arena of at
 * least tcd_bytes() bytes and a HIP stream; like open_stream. */
int tcd_open(int width, int height, const kpd_params* det, const kpd_tcd_params* tp, void* dev_arena,
             size_t arena_bytes, void* hip_stream, kpd_tcd** out);

/* Process the next frame (flags and pitch as push_frame; with
 * KPD_FRAME_DEVICE_RETAIN the frame must stay unchanged until the next
 * push, which matches against it). Asynchronous. */
int tcd_push(kpd_tcd* s, const uint8_t* frame, size_t pitch_bytes, int flags);

/* Copy the current tracks (synchronises): *count receives their number;
 * KPD_ETRUNC, copying nothing, when it exceeds capacity. */
int tcd_get(kpd_tcd* s, kpd_track* out, size_t capacity, size_t* count);

/* Device pointers to the current tracks and their uint32 count, valid until
 * the next push. Does not synchronise. */
int tcd_device_result(kpd_tcd* s, const kpd_track** d_tracks, const uint32_t** d_count);

/* Start a new group with the next frame. */
int tcd_reset(kpd_tcd* s);

/* Wait for the tracker's work and release it (the inner stream too). */
int tcd_close(kpd_tcd* s);

#ifdef __cplusplus
}
#endif
#endif /* KPD_H */
