/*
 * fe.h -- modified no-search (MNS) fractal image encoder for AMD gfx950.
 *
 * C ABI of libfe.so.  Every entry point takes plain pointers and sizes; no
 * C++ or framework types cross it, no exception escapes it, and every call
 * returns an fe_status.  After a failure, fe_last_error() returns a short
 * text for the calling thread.
 *
 * The method is the one of "A Modified No Search Algorithm for Fractal Image
 * Compression" (Salarian, Mohamadinia, Rasekhi):
 *   - an image is cut into B x B range blocks; each range is matched against
 *     the single 2B x 2B domain block with the same centre, reduced to B x B
 *     by the mean of every 2 x 2 pixel group (Sec. 3, Fig. 1b);
 *   - only a contrast s and a luminance are fitted; the range is stored if
 *     its error is below the level's threshold or the level is the last one,
 *     otherwise it is split into four (Sec. 3, quadtree);
 *   - ranges that fail get a second phase (Sec. 3.1 Technique 1, Sec. 3.2):
 *     if every sub-block mean is close to the range mean, each sub-block is
 *     fitted with one of two level-dependent contrasts, and the range is
 *     stored with its mean, three sub-block means (the fourth follows from
 *     eq. (1), Sec. 3.3) and one contrast bit per sub-block;
 *   - decoding iterates the stored contractive maps from any start image
 *     (Sec. 1).
 * The exhaustive search that no-search replaces (Sec. 1: every step-1
 * domain, (W-2B+1)(H-2B+1) candidates per range) is provided as a baseline.
 *
 * Arithmetic.  All encoder arithmetic is exact integer arithmetic.  With
 * n = B^2, Sum r, Sum r^2, Sum d, Sum d^2 and Sum r T_e(d) for the 8 square
 * isometries e, Q = n Sum d^2 - (Sum d)^2, R = n Sum r^2 - (Sum r)^2 and
 * P_e = n Sum r T_e(d) - Sum r Sum d, a phase-1 fit with contrast k/8
 * (k = 0..7) and luminance m (the range mean rounded half up) has the scaled
 * collage error S = k^2 Q - 16 k P_e + 64 R + 64 (n m - Sum r)^2 = 64 n E,
 * E = sum over the block of (prediction - pixel)^2 with prediction
 * (k/8)(T_e(d) - mean d) + m.  The best (e, k) minimises S (lowest e, then
 * lowest k on ties).  A range at level l is accepted when S < 64 n^2 t_l,
 * i.e. its MSE is below the integer threshold t_l.
 *
 * Memory.  Pointers named d_* are device pointers (any HIP allocation on the
 * context's device, e.g. a torch tensor's data_ptr()); h_* are host
 * pointers.  The caller owns every input and output buffer; the library
 * owns only its internal scratch, held by the fe_ctx and released by
 * fe_destroy.  `stream` is a hipStream_t (NULL = the null stream); work is
 * enqueued on it and, unless a call says otherwise, the call returns
 * without waiting.  One fe_ctx must not be used by two threads at once, and
 * calls that share one fe_ctx must be issued on one stream (they share its
 * scratch).
 */
#ifndef FE_H
#define FE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fe_status {
  FE_OK = 0,
  FE_ERR_INVALID = 1,   /* a parameter is out of range or a pointer is NULL */
  FE_ERR_SHAPE = 2,     /* image sides / stride / alignment do not fit the block sizes */
  FE_ERR_CAPACITY = 3,  /* output too small; the needed count is reported */
  FE_ERR_DEVICE = 4,    /* a HIP call failed or no usable gfx950 device */
  FE_ERR_OOM = 5,       /* device or pinned host allocation failed */
  FE_ERR_BUSY = 6       /* a queue or slot limit was reached; retry later */
} fe_status;

/*
 * One stored transform, 16 bytes, little-endian, every byte defined (two
 * equal streams are equal byte for byte).
 *
 *   x, y      range top-left corner in pixels.
 *   dx, dy    domain origin in pixels: for MNS the co-centred origin
 *             clamp(x - B/2, 0, W - 2B) (likewise dy), for the exhaustive
 *             search the chosen step-1 origin (any parity).  A phase-2
 *             record holds the co-centred origin of the whole range; each
 *             of its sub-blocks uses its own co-centred domain of size B.
 *   level     0-based quadtree level: B = b_max >> level.
 *   flags     bit 0 (FE_TRANSFORM_PHASE2): phase-2 record (Sec. 3.1).
 *   iso       phase 1: isometry 0..7 applied to the domain before the fit:
 *             0 identity, 1 mirror left-right, 2 mirror top-bottom,
 *             3 rotate 180, 4 transpose, 5 rotate 90 clockwise,
 *             6 rotate 90 counter-clockwise, 7 anti-transpose
 *             (T_e(d)[i][j] = d[i][j], d[i][B-1-j], d[B-1-i][j],
 *             d[B-1-i][B-1-j], d[j][i], d[B-1-j][i], d[j][B-1-i],
 *             d[B-1-j][B-1-i]).  Phase 2: 0.
 *   s_idx     phase 1: k, contrast s = k/8 (three bits, Sec. 3.3).
 *             Phase 2: bit c set -> sub-block c uses the second contrast of
 *             the level's set {.2,.5}, {.4,.65}, {.5,.9} for levels 1, 2, 3
 *             (Sec. 3.2); sub-blocks c = 0..3 are top-left, top-right,
 *             bottom-left, bottom-right.
 *   lum       phase 1: luminance m, the range mean rounded half up (one
 *             byte, Sec. 3.3).  Phase 2: the range mean O_i.
 *   dlum      phase 2: O_c - O_i for sub-blocks c = 0, 1, 2, within
 *             +-15 at level 1 and +-31 at levels 2 and 3 (5 and 6 bits
 *             with sign, Sec. 3.3); O_3 = 4 O_i - O_0 - O_1 - O_2 (eq. (1)).
 *             Zero in phase 1.
 *
 * A stream lists the transforms of one image in depth-first order: top
 * tiles in raster order, and inside a tile the quadtree in pre-order with
 * children top-left, top-right, bottom-left, bottom-right.
 */
typedef struct fe_transform {
  uint16_t x, y;
  uint16_t dx, dy;
  uint8_t level;
  uint8_t flags;
  uint8_t iso;
  uint8_t s_idx;
  uint8_t lum;
  int8_t dlum[3];
} fe_transform;

#define FE_TRANSFORM_PHASE2 1u

/* fe_params.flags */
#define FE_PHASE2 1u       /* run Technique 1 on ranges that fail (MNS); off = plain no-search */
#define FE_FULL_SEARCH 2u  /* exhaustive step-1 search (Sec. 1) instead of the co-centred domain; no phase 2 */
#define FE_IDENTITY_ONLY 4u /* phase 1 fits the identity isometry only: the stream then fits the paper's
                              14-bit phase-1 code (Sec. 3.3), which stores no isometry; MNS only */
#define FE_LOCAL_SEARCH 8u  /* local search (Sec. 2): the best of the 2B x 2B blocks that contain the range
                              (step 1, (B+1)^2 away from the borders), identity only; no phase 2;
                              same limits as FE_FULL_SEARCH */

/*
 * Encoder parameters.
 *   b_max, b_min  largest and smallest range side: powers of two with
 *                 2 <= b_min <= b_max, 4 <= b_max <= 32 and at most four
 *                 levels (two level bits, Sec. 3.3; the paper's tree is
 *                 16 -> 2).  b_min = 2 is taken by fe_encode,
 *                 fe_encode_batch, plans and the server (MNS or no-search,
 *                 b_max 4, 8 or 16), not by the exhaustive and local
 *                 searches.
 *   n_thr         number of thresholds = L - 1, L = log2(b_max/b_min) + 1.
 *   flags         FE_PHASE2, FE_FULL_SEARCH, FE_IDENTITY_ONLY (MNS only),
 *                 FE_LOCAL_SEARCH (not with FE_FULL_SEARCH).
 *   mse_thr[l-1]  integer MSE threshold t_l of level l = 1..L-1 (the last
 *                 level is always stored, Sec. 3); unused entries ignored.
 */
typedef struct fe_params {
  uint32_t b_max;
  uint32_t b_min;
  uint32_t n_thr;
  uint32_t flags;
  uint32_t mse_thr[4];
} fe_params;

/* One image of a batch: device pointer, sides, row pitch in bytes. */
typedef struct fe_image_desc {
  const uint8_t* data;
  uint32_t width;
  uint32_t height;
  uint32_t stride;
  uint32_t reserved; /* must be 0 */
} fe_image_desc;

typedef struct fe_ctx fe_ctx;

/* Text of the last failure on this thread ("" if none).  Valid until the
 * thread's next fe_* call. */
const char* fe_last_error(void);

/* Static name of a status code. */
const char* fe_status_string(fe_status status);

/* Library ABI version (major * 10000 + minor * 100 + patch). */
int fe_version(void);

/*
 * Host-only check of an encode request (no device needed).  FE_ERR_INVALID
 * for bad block sizes, thresholds count or flags; FE_ERR_SHAPE when W or H
 * is not a multiple of b_max, smaller than 2 b_max (the domain of every
 * range must fit), larger than 65536, or stride < W, or stride not a
 * multiple of 4.
 */
fe_status fe_validate(uint32_t width, uint32_t height, uint32_t stride, const fe_params* params);

/* Upper bound of the stream length of one W x H image:
 * (W / b_min) * (H / b_min); 0 if b_min is 0. */
size_t fe_max_transforms(uint32_t width, uint32_t height, uint32_t b_min);

/*
 * Open a context on HIP device `device` (must be gfx950).  FE_ERR_DEVICE
 * when there is no such device.  The context owns scratch memory that grows
 * with the largest request seen and is freed by fe_destroy.  Calls on one
 * context share that scratch: issue them from one host thread; calls on
 * different streams are ordered through it (a later call waits on the device
 * for the image table and block descriptors an earlier one wrote) but their
 * kernels must not overlap.  A batch with the same image table as the
 * previous call (same images, sizes and tile shape) reuses the table and
 * block descriptors already on the device.
 */
fe_status fe_create(int device, fe_ctx** out);
void fe_destroy(fe_ctx* ctx);

/*
 * Domain pyramid level used by no-search (Sec. 3: each domain pixel is the
 * mean of a 2 x 2 pixel group): d_out[j * (W/2) + i] = (I[2j][2i] + I[2j][2i+1] +
 * I[2j+1][2i] + I[2j+1][2i+1] + 2) >> 2, a dense (H/2) x (W/2) uint8 image.
 * W and H even and >= 2; stride >= W, multiple of 4; d_img 4-byte aligned.
 */
fe_status fe_downsample(fe_ctx* ctx, const uint8_t* d_img, uint32_t width, uint32_t height,
                        uint32_t stride, uint8_t* d_out, void* stream);

/*
 * Moments of explicit ranges against their co-centred domains (the moment
 * step of Sec. 3).  Range i of side `block` (4, 8, 16 or 32) has top-left
 * corner x = d_xy[i] & 0xffff, y = d_xy[i] >> 16 (multiples of `block`,
 * inside the image); the image must satisfy fe_validate for b_max = block.
 * Writes 12 uint32 per range to d_moments[12 i ..]: Sum r, Sum r^2, Sum d,
 * Sum d^2, then Sum r T_e(d) for e = 0..7, where d is the domain reduced to
 * block x block.  Out-of-image ranges give FE_ERR_INVALID before any launch
 * only if detectable on the host; the device skips them (moments left 0).
 */
fe_status fe_range_moments(fe_ctx* ctx, const uint8_t* d_img, uint32_t width, uint32_t height,
                           uint32_t stride, uint32_t block, const uint32_t* d_xy, uint32_t count,
                           uint32_t* d_moments, void* stream);

/*
 * Encode one image (MNS, Sec. 3 and 3.1-3.3; or the exhaustive baseline
 * with FE_FULL_SEARCH).  d_img is W x H uint8 with row pitch `stride`
 * bytes (4-byte aligned).  Writes the stream to d_out[0 .. *n_out).
 * With b_min = 2 the 2 x 2 ranges take their co-centred domains at odd
 * origins (x - 1): the tree runs down to 4 x 4 as usual, and the 2 x 2
 * level follows in a second kernel that forms those domains' means from the
 * pixels; same stream format.
 * Waits for the stream to finish (the count is needed on the host).
 * FE_ERR_CAPACITY if cap is smaller than the stream; *n_out then holds
 * the needed count and d_out is left unspecified.  cap =
 * fe_max_transforms(W, H, b_min) always suffices.
 */
fe_status fe_encode(fe_ctx* ctx, const uint8_t* d_img, uint32_t width, uint32_t height,
                    uint32_t stride, const fe_params* params, fe_transform* d_out, size_t cap,
                    size_t* n_out, void* stream);

/*
 * Encode a batch of images of any sides in one pass (MNS, Sec. 3 and
 * 3.1-3.3, for every image of the list; one launch covers every range of
 * every image).  Image k's stream is written to
 * d_out[d_offsets[k] .. d_offsets[k+1]); d_offsets (device, n_imgs + 1
 * entries) is written by the device.  If n_out is not NULL the call waits
 * and stores the total count (FE_ERR_CAPACITY as for fe_encode); if it is
 * NULL the call returns at once and the caller must check
 * d_offsets[n_imgs] <= cap itself (entries beyond cap are not written).
 * FE_FULL_SEARCH is not accepted here.  Trees down to 2 x 2 address record
 * slots in 32 bits: a batch needing 2^32 slots or more gives FE_ERR_SHAPE.
 */
fe_status fe_encode_batch(fe_ctx* ctx, const fe_image_desc* h_imgs, uint32_t n_imgs,
                          const fe_params* params, fe_transform* d_out, size_t cap,
                          uint64_t* d_offsets, size_t* n_out, void* stream);

/*
 * For callers that cannot allocate device memory during the call: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The same MNS encode as fe_encode (same kernels, same stream),
 * with every scratch buffer taken from a static device array of 32 MiB per
 * GPU, held by the library until the process ends; the call makes no device
 * or host allocation and copies nothing from the host (its image entry is
 * written by a kernel).  The stream goes to d_out[0 .. d_offsets[1]);
 * d_offsets (device, 2 entries, 8-byte aligned) receives 0 and the stream
 * length.  If n_out is not NULL the call waits and stores the length
 * (FE_ERR_CAPACITY as for fe_encode); if it is NULL it returns at once and
 * the caller checks d_offsets[1] <= cap (entries beyond cap are not
 * written).  An image whose scratch (about W*H bytes at b_min = 4, 5 W*H at
 * b_min = 2, plus tile masks and descriptors) exceeds the 32 MiB gives
 * FE_ERR_CAPACITY before any launch.  MNS and no-search only
 * (FE_FULL_SEARCH / FE_LOCAL_SEARCH: FE_ERR_INVALID).  Every call on one GPU
 * shares that GPU's array, which keeps the last call's contents: calls that
 * overlap on one GPU (on different streams, threads or contexts) race.
 */
fe_status fe_encode_noalloc(fe_ctx* ctx, const uint8_t* d_img, uint32_t width, uint32_t height,
                            uint32_t stride, const fe_params* params, fe_transform* d_out, size_t cap,
                            uint64_t* d_offsets, size_t* n_out, void* stream);

/*
 * Recorded batch encode (a HIP graph).  fe_plan_create validates the batch
 * as fe_encode_batch does, allocates the plan's own scratch (record slots
 * and masks for every top tile, block descriptors, ordering scratch),
 * uploads the image table, builds the workgroup block descriptors (they
 * depend only on the images' addresses and sizes) and records the launch
 * sequence once.
 * fe_plan_launch replays it on `stream`: the images are re-read in place
 * (their contents may change between launches, their addresses and sizes
 * may not), and the stream and offsets are written to d_out / d_offsets as
 * fe_encode_batch writes them; the caller reads d_offsets[n_imgs] and checks
 * it against cap.  Launches on one plan must not overlap; fe_plan_destroy
 * waits for the device.  The plan keeps the context's tile shape at
 * creation.  If timing (fe_timing_enable) is on when the plan is created,
 * the graph also holds event nodes, and each launch made while timing is on
 * times its encode and ordering kernels into the context as eager calls
 * do.  The context must outlive the plan.  For callers that encode the same set of buffers repeatedly
 * (video frames, a fixed input ring).
 */
typedef struct fe_plan fe_plan;
fe_status fe_plan_create(fe_ctx* ctx, const fe_image_desc* h_imgs, uint32_t n_imgs,
                         const fe_params* params, fe_transform* d_out, size_t cap,
                         uint64_t* d_offsets, fe_plan** out);
fe_status fe_plan_launch(fe_plan* plan, void* stream);
void fe_plan_destroy(fe_plan* plan);

/*
 * Decode (Sec. 1): start from d_start (W x H, dense) or mid-grey 128 if
 * d_start is NULL, and apply the n transforms `iters` times; every
 * iteration computes all pixels from the previous iterate (Jacobi).  A
 * phase-1 transform writes, for each pixel p of its range,
 *   clamp(floor((k (n d_p - Sum d) + 8 n m + 4 n) / (8 n)), 0, 255),
 * with d the 2 x 2 round-half-up means of the current iterate over the 2B x
 * 2B block at (dx, dy), taken under the isometry; a phase-2 transform does
 * the same for each sub-block with contrast c/20, its own co-centred domain
 * and luminance O_c.  The stream must tile the image; pixels it does not
 * cover keep the start value.  Writes the W x H result to d_out (dense).
 * Checks every transform on the device first and returns FE_ERR_INVALID
 * (and leaves d_out unspecified) if one is out of range; waits for that
 * check.
 */
fe_status fe_decode(fe_ctx* ctx, const fe_transform* d_t, size_t n, uint32_t width,
                    uint32_t height, uint32_t b_max, uint32_t iters, const uint8_t* d_start,
                    uint8_t* d_out, void* stream);

/*
 * Two decoders compute the same iterate bit for bit.  The tile decoder
 * reduces the iterate to its 2 x 2 means once per 128 x 128-pixel block in
 * LDS and writes four pixels per lane; it runs when W and H are multiples
 * of b_max (each at least 2 b_max), d_out is 4-byte aligned, and the stream
 * lists the tiles in raster order with each tile's transforms partitioning
 * it in Morton order (the order fe_encode writes) with co-centred domains
 * (Sec. 3.1), and its plan (2.3 KB per 64 x 64-pixel block, kept in the
 * context) can be allocated; the 2 x 2 pieces of such a stream (2 x 2
 * ranges, phase-2 transforms of side 4) are decoded beside it by a kernel
 * of their own each iteration.  The record decoder (one wave per transform)
 * runs any valid stream.  fe_decode_set_mode selects FE_DECODE_AUTO (the default: tiles
 * when allowed) or FE_DECODE_RECORDS for a context; fe_decode_last returns
 * FE_DECODE_TILES or FE_DECODE_RECORDS for the last fe_decode on ctx.
 */
enum { FE_DECODE_AUTO = 0, FE_DECODE_RECORDS = 1, FE_DECODE_TILES = 2 };
fe_status fe_decode_set_mode(fe_ctx* ctx, int mode);
int fe_decode_last(const fe_ctx* ctx);

/*
 * Zoom decoding (Sec. 1: the stored maps do not depend on the resolution).
 * Decodes a stream encoded for a W x H image (top blocks b_max) at `zoom`
 * times the size: every transform's range and domain origins are multiplied
 * by zoom and the maps are iterated on a zoom W x zoom H image with top blocks
 * of zoom b_max, as fe_decode does (same arithmetic, same choice between the
 * two decoders; a co-centred domain stays co-centred).  zoom is a power of
 * two with zoom * b_max <= 32 (1 decodes at the native size); zoom W and
 * zoom H are at most 65536.  d_start (or mid-grey when NULL) and d_out are
 * zoom W x zoom H, dense.  The transforms are checked against the native
 * W x H image first (FE_ERR_INVALID as in fe_decode); the zoomed copy lives
 * in the context (16 bytes per transform).  Waits for the check.
 */
fe_status fe_decode_zoom(fe_ctx* ctx, const fe_transform* d_t, size_t n, uint32_t width,
                         uint32_t height, uint32_t b_max, uint32_t zoom, uint32_t iters,
                         const uint8_t* d_start, uint8_t* d_out, void* stream);

/*
 * The compressed file (Sec. 3.3; Technique 2, Sec. 3.4).  A 64-bit header
 * (W - 1 and H - 1 in 16 bits each, log2 b_max and log2 b_min in 3 bits
 * each, the isometry flag in 1 bit, 25 zero bits) is followed by one code
 * per transform in stream order.  Bits are numbered from the least
 * significant bit of byte 0 upwards and every field is written least
 * significant bit first.  A code is: the phase bit (1 = phase 2); the
 * 0-based level in 2 bits, left out for a block of the last level that is
 * not the top-left child of its parent (Technique 2); the luminance byte
 * (m, or O_i in phase 2); then, in phase 1, the contrast k in 3 bits and,
 * with FE_PACK_ISOMETRY, the isometry in 3 bits (14 or 17 bits in all); in
 * phase 2, O_c - O_i for c = 0, 1, 2 as M-bit sign (1 = negative) and
 * magnitude, M = 5 at level 1 and 6 below, then the 4 contrast bits (30 or
 * 33 bits).  No domain position is stored: the decoder places each block at
 * the next free cell of the depth-first walk and gives it its co-centred
 * domain (Sec. 3).
 *
 * fe_pack writes the file of one image's stream (d_t, n transforms, as
 * fe_encode returns it) to d_out (device, 8-byte aligned, cap bytes; the
 * file takes ceil(bits / 64) * 8 bytes, zero-padded) and its exact length
 * in bits to *n_bits.  The stream must be in encoder order with co-centred
 * domains, and W, H multiples of b_max (FE_ERR_INVALID otherwise, as for
 * fields a code cannot hold: phase-2 differences beyond +-(2^(M-1) - 1), or
 * an isometry other than the identity without FE_PACK_ISOMETRY, which the
 * encoder's FE_IDENTITY_ONLY guarantees).  FE_ERR_CAPACITY if cap is too
 * small.  Waits for the stream.  fe_pack_bound gives a cap that always
 * suffices for n transforms.
 *
 * fe_unpack (host only, no device) parses a file of n_bits bits back into
 * transforms (h_out, cap; co-centred dx, dy filled in) and the header's
 * fields (*info).  FE_ERR_INVALID for a malformed file (truncated, a level
 * out of range, a block that does not fit the next free cell);
 * FE_ERR_CAPACITY if cap is too small, with *n_out set to the number needed.
 */
#define FE_PACK_ISOMETRY 1u
typedef struct fe_stream_info {
  uint32_t width, height, b_max, b_min, flags;
} fe_stream_info;
size_t fe_pack_bound(size_t n);
fe_status fe_pack(fe_ctx* ctx, const fe_transform* d_t, size_t n, uint32_t width, uint32_t height,
                  uint32_t b_max, uint32_t b_min, uint32_t flags, uint8_t* d_out, size_t cap,
                  uint64_t* n_bits, void* stream);
fe_status fe_unpack(const uint8_t* h_bits, uint64_t n_bits, fe_transform* h_out, size_t cap, size_t* n_out,
                    fe_stream_info* info);

/*
 * Exhaustive search of explicit ranges (Sec. 1): for each range of side
 * `block` (4, 8 or 16) at d_xy[i] (x | y << 16, multiples of block), find
 * the best of all (W - 2B + 1)(H - 2B + 1) step-1 domains, 8 isometries and
 * contrasts k/8 (minimum S, then lowest domain index v * (W - 2B + 1) + u,
 * then lowest isometry, then lowest k).  Writes 4 uint32 per range:
 * domain index, e | k << 8 | m << 16, and S as low / high 32-bit words.
 * The image must satisfy fe_validate for b_max = block, and the number of
 * domain origins must be below 2^20 (FE_ERR_SHAPE otherwise).  fe_encode
 * with FE_FULL_SEARCH runs the same search inside the quadtree (b_max <=
 * 16); its records hold the chosen domain origin in dx, dy.
 */
fe_status fe_full_search_ranges(fe_ctx* ctx, const uint8_t* d_img, uint32_t width, uint32_t height,
                                uint32_t stride, uint32_t block, const uint32_t* d_xy, uint32_t count,
                                uint32_t* d_out, void* stream);

/*
 * Tile shapes of the fused encode kernel.  A workgroup runs the quadtrees of
 * a gx x gy block of top-level tiles (b_max x b_max each); the shape trades
 * LDS per workgroup (occupancy) against the halo of domain pixels staged
 * around the block.  fe_tile_shapes lists the shapes built for (b_max,
 * b_min) (first = default) and returns their number (at most max_out
 * written).  fe_set_tile_shape selects one for a context (gx = gy = 0
 * restores the default); FE_ERR_INVALID if the shape is not built.  With
 * no shape set, an encode call whose tiles would fill fewer than 256
 * default-shape workgroups (one per compute unit) takes the shape with the
 * fewest tiles per workgroup.  The encoded stream does not depend on the
 * shape.
 */
int fe_tile_shapes(uint32_t b_max, uint32_t b_min, uint32_t* gx, uint32_t* gy, int max_out);
fe_status fe_set_tile_shape(fe_ctx* ctx, uint32_t b_max, uint32_t b_min, uint32_t gx, uint32_t gy);
fe_status fe_get_tile_shape(fe_ctx* ctx, uint32_t b_max, uint32_t b_min, uint32_t* gx, uint32_t* gy);

/*
 * Autotuner: encode the given batch (as fe_encode_batch, into the caller's
 * d_out / d_offsets) `reps` times with every built tile shape for
 * (b_max, b_min), in two rounds over the shapes, time the fused kernel with
 * HIP events on `stream`, and select the shape with the least mean kernel
 * time (the better of its two rounds) for this context.  Writes the chosen
 * shape and that time in milliseconds.  Waits for the device.
 */
fe_status fe_autotune(fe_ctx* ctx, const fe_image_desc* h_imgs, uint32_t n_imgs, const fe_params* params,
                      fe_transform* d_out, size_t cap, uint64_t* d_offsets, uint32_t reps, uint32_t* gx,
                      uint32_t* gy, double* ms, void* stream);

/*
 * Encode server (continuous batching).  The server's parameter set fixes
 * the block sizes (b_max, b_min: the kernel it runs); each request may bring
 * its own thresholds and FE_PHASE2 / FE_IDENTITY_ONLY flags.
 *
 * fe_server_create: device memory of `hbm_budget` bytes (a quarter holds
 * per-tile record slots and masks, the rest images and ordering scratch)
 * and `host_budget` bytes of pinned host memory for inputs and results are
 * reserved up front; at most `max_slots` requests are admitted at once; one
 * step launches the fused kernel over at most `step_blocks` workgroup blocks
 * of top tiles drawn first-come first-served from all admitted requests.
 * A worker thread drives the steps.  The ordering kernel writes a finished
 * request's records straight into its pinned result buffer, which stays
 * reserved until the request is fetched: callers should poll promptly.
 * Creation also makes one host-to-device copy of each size class on each
 * of the server's streams (tens of milliseconds in all), so that no step
 * pays the runtime's set-up of a copy path; FE_ERR_DEVICE if that fails.
 *
 * fe_server_submit copies the host image (W x H, row pitch `stride`) into
 * pinned staging and queues it; the caller may reuse h_img on return.
 * `params` (copied; NULL = the server's) are the request's encoder
 * parameters: b_max and b_min must equal the server's and flags may hold
 * FE_PHASE2 and FE_IDENTITY_ONLY only (FE_ERR_INVALID otherwise); requests
 * with different parameters share steps.
 * FE_ERR_BUSY when the pinned staging is full (retry later), FE_ERR_OOM
 * when the request can never fit the device budget, FE_ERR_SHAPE /
 * FE_ERR_INVALID as fe_validate.  Requests are admitted in arrival order
 * when their device footprint fits.
 *
 * fe_server_submit_pinned queues an image that already lies in pinned
 * host memory (hipHostMalloc or equivalent; FE_ERR_INVALID otherwise) and
 * copies it to the device straight from there, with no host-side copy: the
 * caller must keep h_img unchanged until the request is done.
 *
 * fe_server_poll: *done = 0 while the request runs.  When done, *n is the
 * stream length and *latency_ms the time from submit to the records being
 * in host memory; if h_out is not NULL the stream is copied there (cap >=
 * *n, else FE_ERR_CAPACITY and nothing is released) and the request is
 * released (its id becomes unknown).  A request that failed on the device
 * returns FE_ERR_DEVICE and is released.  The stream equals fe_encode's for
 * the same image and the request's parameters, whatever else (and with
 * whatever parameters) was in flight.
 *
 * fe_server_wait blocks up to `timeout_us` microseconds for a request to
 * finish (done or failed) and returns its id, each finished id once, in
 * completion order; FE_ERR_BUSY if none finished in time.  An id fetched by
 * fe_server_poll before it was reported is not reported.
 *
 * fe_server_destroy stops the worker, waits for the device and frees
 * everything, including unfetched results.  Submit / poll / stats may be
 * called from several threads.
 */
typedef struct fe_server fe_server;

fe_status fe_server_create(int device, const fe_params* params, size_t hbm_budget, size_t host_budget,
                           uint32_t max_slots, uint32_t step_blocks, fe_server** out);
fe_status fe_server_submit(fe_server* server, const uint8_t* h_img, uint32_t width, uint32_t height,
                           uint32_t stride, const fe_params* params, uint64_t* req);
fe_status fe_server_submit_pinned(fe_server* server, const uint8_t* h_img, uint32_t width, uint32_t height,
                                  uint32_t stride, const fe_params* params, uint64_t* req);
fe_status fe_server_poll(fe_server* server, uint64_t req, fe_transform* h_out, size_t cap, size_t* n,
                         int* done, double* latency_ms);
fe_status fe_server_wait(fe_server* server, uint32_t timeout_us, uint64_t* req);
/*
 * Zero-copy access to a finished request's records: *recs points at its
 * *n records (stream order, as fe_server_poll would copy them) in the
 * server's pinned host memory, and stays valid until
 * fe_server_release(server, req), which frees them and forgets the id.
 * FE_ERR_BUSY while the request runs; FE_ERR_DEVICE (request released) if
 * it failed; FE_ERR_INVALID for an unknown id.  A request is released either
 * by fe_server_poll with h_out or by fe_server_release, not both.
 */
fe_status fe_server_result(fe_server* server, uint64_t req, const fe_transform** recs, size_t* n,
                           double* latency_ms);
fe_status fe_server_release(fe_server* server, uint64_t req);
/*
 * Where a request's latency went (execution; no passage of the paper): the
 * times, in milliseconds after its submission, at which request `req` was
 * admitted (its image copy issued), had its first and its last step
 * launched, and was found complete, written to ms[0 .. min(n, 4)).  The
 * request must be done and not yet fetched (FE_ERR_BUSY otherwise;
 * FE_ERR_INVALID for an unknown id).
 */
fe_status fe_server_request_times(fe_server* server, uint64_t req, double* ms, uint32_t n);
fe_status fe_server_stats(fe_server* server, uint64_t* steps, uint64_t* blocks, uint64_t* completed,
                          size_t* hbm_used, uint32_t* in_flight, uint32_t* queued);
void fe_server_destroy(fe_server* server);

/*
 * Kernel timing.  While enabled, each launch of the library's main kernels
 * (below) is bracketed by HIP events recorded on the launch's own stream.
 * fe_timing_read waits for those events, adds each kernel's event-to-event
 * time (milliseconds) and launch count into ms[k] / launches[k] for
 * k < n (n <= FE_TIMING_SLOTS), and clears them.  At most 4096 launches are
 * held between reads; later ones are not timed.  Enabling timing adds an
 * event record before and after each timed launch and nothing else.
 */
#define FE_TIMING_ENCODE 0      /* fused MNS quadtree kernel */
#define FE_TIMING_SCATTER 1     /* stream-order kernel */
#define FE_TIMING_DECODE 2      /* one decoder iteration */
#define FE_TIMING_FULLSEARCH 3  /* exhaustive-search GEMM + argmin */
#define FE_TIMING_SLOTS 8

fe_status fe_timing_enable(fe_ctx* ctx, int enable);
fe_status fe_timing_read(fe_ctx* ctx, double* ms, uint64_t* launches, uint32_t n);
/*
 * Which slots are timed while timing is on: bit k of slot_mask for slot k
 * (default: all).  Each timed launch costs two event records on the GPU
 * (a few microseconds each), so a caller that needs one kernel's time can
 * leave the others untimed.  Applies to eager launches; a recorded plan
 * created with timing on times its encode and ordering kernels.
 */
fe_status fe_timing_select(fe_ctx* ctx, uint32_t slot_mask);

#ifdef __cplusplus
}
#endif

#endif /* FE_H */
