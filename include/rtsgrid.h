/*
 * rtsgrid: convolutional gridding and degridding of radio visibilities on AMD
 * MI355X (gfx950).  C ABI of librtsgrid.so.
 *
 * What is computed (Edgar et al., "Enabling a High Throughput Real Time Data
 * Pipeline for a Large Radio Telescope Array with GPUs", Section 5, Eq. (1)):
 * every visibility V_i at (u_i, v_i) is convolved with a compact gridding
 * function and added onto a regular uv grid,
 *     G[c][y][x] = sum_i w_i V_i k(y - y_i) k(x - x_i),
 * where k is a Kaiser-Bessel window of support W cells sampled at OS phases per
 * cell (the nearest phase is used) and k vanishes at and beyond W/2.  Degridding
 * is the adjoint without weights,
 *     M_i = sum_{x,y} k(y - y_i) k(x - x_i) G[c][y][x].
 * Coordinates: x_i = u_i f_c / (c du) + N/2 cells (pixel N/2 is u = 0), snapped to
 * 1/OS cell by rounding half up, xs = floor(x OS + 1/2), every product and sum
 * rounded once in FP64 (no fused multiply-add), so the snapped coordinates equal
 * those of a plain IEEE evaluation bit for bit; this is the only FP64 arithmetic besides the
 * accumulators and chi-squared sums, the rest is FP32 (or the matrix-core forms
 * of rts_precision).  A sample is valid iff its weight (at plan time) is non-zero
 * and every tap lies on the grid; invalid samples contribute nothing and predict 0.
 *
 * Layouts (row-major, C-contiguous):
 *   uvw      double  [B][T][3]   metres, device memory
 *   freq_hz  double  [C]         host memory
 *   vis, model       [C][B][T]   complex64 as interleaved float (re, im), device
 *   weights  float   [C][B][T]   device; 0 marks a flagged sample
 *   grid             [C][N][N]   complex64 as interleaved float, [channel][v][u], device
 * A baseline's T time samples are contiguous: the tiled kernels read each
 * baseline's track as one run.
 *
 * Ownership: the caller owns every buffer passed in; a plan owns its own
 * workspace (kernel table, per-sample packed coordinates, the tile-sorted work
 * list).  uvw and weights may be freed once rts_grid_plan has returned AND its
 * stream has been synchronised.
 *
 * Errors: every entry point returns an rts_status and never aborts.  Arguments
 * are validated on the host before any HIP call.  On failure the message is
 * available from rts_last_error() (thread-local).  NaN or Inf in vis / weights
 * propagate; NaN or Inf in uvw make the sample invalid.
 *
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  All calls
 * enqueue asynchronously on it, except: rts_grid_plan synchronises it (once, to
 * size the work list); rts_plan_get_info waits for the last re-plan's counts;
 * the first rts_image call of a plan builds its FFT plan and correction table
 * (allocation and a synchronous copy); the first rts_plan_set_baseline_kernels
 * call allocates the per-baseline tables; rts_autotune_tile times on the stream;
 * rts_plan_destroy waits for the device.
 * One plan must not be used concurrently on two streams.
 */
#ifndef RTSGRID_H
#define RTSGRID_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rts_plan_s *rts_plan_t;
typedef struct rts_graph_s *rts_graph_t;

typedef enum {
  RTS_OK = 0,
  RTS_E_INVALID = 1,      /* bad argument (null pointer, size out of range, ...) */
  RTS_E_NOMEM = 2,        /* device or host allocation failed */
  RTS_E_HIP = 3,          /* a HIP runtime call failed */
  RTS_E_UNSUPPORTED = 4,  /* valid request the library does not implement */
} rts_status;

typedef enum {
  RTS_PREC_FP32 = 0,    /* FP32 arithmetic, FP64 tile accumulation (all entry points) */
  RTS_PREC_BF16X3 = 1,  /* rts_grid and rts_degrid on the matrix cores (Eq. (1) and its adjoint
                           per 16x16-cell subtile): gridding is the contraction Av^T diag(wV) Au
                           over the subtile's samples, degridding H = Av G_subtile followed by the
                           k_x sum, with per-region partial values added to the model with FP32
                           atomics.  Operands are split into BF16 hi+lo (hi*hi + hi*lo + lo*hi,
                           FP32 accumulation; ~16 significant bits per operand; relative error a
                           few 1e-6).  The plan's tile (a multiple of 16 cells) is split into
                           regions of one or two 16x16 subtiles, one wave each.  Supports up to
                           24; per-baseline kernels (rts_plan_set_baseline_kernels).  The fused
                           step runs the same two kernels (degrid, then grid of w (V - M)). */
  RTS_PREC_FP32_MFMA = 2  /* as RTS_PREC_BF16X3, with FP32 operands (v_mfma_f32_16x16x4_f32,
                           FP32 accumulation; relative error ~1e-7) */
} rts_precision;

typedef enum {
  RTS_SCHEDULE_AUTO = 0,        /* the library's choice (currently RTS_SCHEDULE_TILES)          */
  RTS_SCHEDULE_TILES = 1,       /* one workgroup per (channel, tile), XCD-grouped               */
  RTS_SCHEDULE_PERSISTENT = 2   /* two to six workgroups per compute unit pull tiles from eight
                                   per-XCD queues in longest-first order, which the plan builds
                                   (load balance for skewed uv coverage; not in the paper)     */
} rts_schedule;

typedef struct {
  int32_t n_grid;       /* N: grid edge in cells, even, 16 <= N <= 8192                  */
  int32_t support;      /* W: taps per axis, 2 <= W <= 16 (matrix-core plans: <= 24)      */
  int32_t oversample;   /* OS: kernel phases per cell, 1 <= OS <= 64                     */
  int32_t n_chan;       /* C >= 1                                                         */
  int32_t n_base;       /* B >= 1                                                         */
  int32_t n_time;       /* T >= 1; C*B*T*(1+conjugate) < 2^31 and B*T < 2^29            */
  double cell_lambda;   /* du > 0: uv cell size in wavelengths                           */
  double beta;          /* Kaiser-Bessel shape; <= 0 selects 2.34 * W                     */
  int32_t conjugate;    /* 1: also grid conj(w V) at (-u, -v) (rts_grid only)             */
  int32_t tile;         /* uv tile edge in cells: even, divides N, >= W+1, <= 64; 0 = choose
                           (matrix-core plans: also a multiple of 16)                     */
  int32_t precision;    /* rts_precision                                                 */
  int32_t schedule;     /* rts_schedule: how the FP32 tile kernels are launched           */
} rts_params;

typedef struct {
  int64_t n_samples;    /* C*B*T                                                         */
  int64_t n_valid;      /* samples with w != 0 and all taps on the grid                   */
  int64_t n_flagged;    /* samples with w == 0                                            */
  int64_t n_offgrid;    /* samples with w != 0 but a tap off the grid (or non-finite uvw) */
  int64_t n_segments;   /* runs of one baseline's samples sharing a (W+1)^2 cell window   */
  int64_t n_listings;   /* (segment, tile) pairs in the work list                        */
  int64_t n_dropped;    /* listings beyond the work-list capacity after rts_plan_update
                           (non-zero: results are incomplete, build a new plan)          */
  int64_t workspace_bytes;
  int32_t tile;         /* tile edge chosen                                               */
  int32_t seg_max;      /* most samples per segment                                       */
} rts_plan_info;

/*
 * Build a gridding plan (Section 5.2: visibilities are binned by uv tile and each
 * tile's work is listed, so that one workgroup owns each tile of the output).
 * From uvw, the channel frequencies and the weights it computes every sample's
 * snapped FP64 coordinates, groups each baseline's consecutive samples into
 * segments, and sorts the segments by (channel, tile) with a counting sort.
 * Synchronises `stream` once.  *out receives the plan (NULL on failure).
 */
rts_status rts_grid_plan(rts_plan_t *out, const rts_params *params, const double *uvw_m,
                         const double *freq_hz, const float *weights, void *stream);

/* Re-plan in place for a new cadence with the same shape (new uvw and weights):
 * recomputes coordinates, segments and the tile-sorted work list into the plan's
 * existing workspace.  Allocates nothing and does not synchronise, so a whole
 * cadence (update, then grid/degrid calls) can be enqueued back to back.  The
 * work list keeps the capacity sized at rts_grid_plan (+1/8 headroom); listings
 * beyond it are dropped and counted in rts_plan_info.n_dropped, which
 * rts_plan_get_info reports (synchronising the device). */
rts_status rts_plan_update(rts_plan_t plan, const double *uvw_m, const float *weights, void *stream);

/* Eq. (1): grid[c] = sum_i w_i V_i k k over valid samples (and conj(w V) at -uv
 * when the plan was built with conjugate=1).  `grid` [C][N][N] is overwritten. */
rts_status rts_grid(rts_plan_t plan, const float *vis, const float *weights, float *grid,
                    void *stream);

/* Adjoint of Eq. (1) without weights: vis_out[c][b][t] = sum k k G at the +uv
 * position of each valid sample, 0 for invalid samples.  All C*B*T entries are
 * written. */
rts_status rts_degrid(rts_plan_t plan, const float *grid, float *vis_out, void *stream);

/* Fused residual step (Eq. (1) and its adjoint, composed as one model-fitting
 * iteration): M = degrid(grid_in); r = V - M (0 where invalid);
 * grid_out = grid(r, w); chi2 = sum_i w_i |r_i|^2 (FP64).  model_out (C*B*T
 * complex64) and chi2_out (one double in device memory) may be NULL, except that
 * matrix-core plans need model_out (RTS_E_INVALID otherwise).  grid_in and
 * grid_out must not overlap, nor may model_out overlap any other buffer
 * (RTS_E_INVALID).  FP32 plans run one tile kernel; matrix-core plans run their
 * degridding into model_out, then their gridding of w (V - M), which also forms
 * the chi2 partial sums, then one reduction.  Plans built with conjugate=1 return
 * RTS_E_UNSUPPORTED. */
rts_status rts_grid_degrid(rts_plan_t plan, const float *vis, const float *weights,
                           const float *grid_in, float *model_out, float *grid_out,
                           double *chi2_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): rts_grid_plan followed
 * by rts_grid_degrid in one call, with the plan's workspace carved from a static
 * device array of the library (64 MiB per device, held until the process ends)
 * instead of allocated.  Same arguments and results as those two calls for an
 * FP32 plan (params->precision RTS_PREC_FP32, conjugate 0, support <= 16,
 * schedule ignored: one workgroup per (channel, tile)); freq_hz is host memory,
 * every other buffer device memory owned by the caller.  The work list is sized
 * for the worst case (four listings per sample), so nothing is dropped.  Returns
 * RTS_E_INVALID with a message naming the bytes needed when the problem does not
 * fit the static array (about 34 bytes per sample plus 20 per (channel, tile)
 * pair; the benchmark-sized problems do not fit: use rts_grid_plan +
 * rts_grid_degrid there).  Calls no hipMalloc, hipFree or allocating library
 * routine and does not synchronise; its kernel table and per-channel scales
 * reach the device as kernel arguments.  Every call on one device shares that
 * device's array, so calls that overlap on one device (on different streams, or
 * from several threads) race: serialise them.  Each call re-initialises what it
 * reads from the array. */
rts_status rts_grid_degrid_noalloc(const rts_params *params, const double *uvw_m, const double *freq_hz,
                                   const float *weights, const float *vis, const float *grid_in, float *model_out,
                                   float *grid_out, double *chi2_out, void *stream);

/* Backward of gridding, for automatic differentiation of Eq. (1): with D the
 * plan's degridding (the adjoint of its gridding without weights),
 *     grad_vis     = w * D(grad_grid)                    (complex, [C][B][T])
 *     grad_weights = Re(conj(vis) * D(grad_grid))         (float,   [C][B][T])
 * in PyTorch's convention for complex gradients (dL/dRe + i dL/dIm); both are 0 at
 * samples the plan does not grid.  grad_grid: complex64 [C][N][N], the gradient
 * with respect to the plan's grid output.  grad_vis is required (it also holds
 * D(grad_grid) while the weight term is formed); grad_weights may be NULL.  Device
 * buffers, caller-owned; grad_vis and grad_weights must not overlap each other or
 * the inputs.  Asynchronous on `stream`; allocates nothing.
 * Errors: RTS_E_UNSUPPORTED for plans built with conjugate=1 (their gridding also
 * adds conj(w V), which is not complex-linear in V), RTS_E_INVALID, RTS_E_HIP. */
rts_status rts_grid_backward(rts_plan_t plan, const float *vis, const float *weights, const float *grad_grid,
                             float *grad_vis, float *grad_weights, void *stream);

/* Backward of the chi-squared of the fused step, chi2 = sum_i w_i |vis_i - model_i|^2
 * over the plan's valid samples, with model = D(grid_in).  From the model and the
 * grid the fused step wrote (grid_resid = D^T(w r), r = vis - model at valid
 * samples, 0 elsewhere) and the upstream gradient g = dL/dchi2 (one double in
 * device memory):
 *     grad_vis = 2 g w r,   grad_weights = g |r|^2,   grad_grid = -2 g grid_resid
 * (PyTorch's convention for complex gradients).  Each output may be NULL; buffers
 * are device memory, caller-owned, outputs must not overlap the inputs
 * (grad_grid may be grid_resid itself).  Asynchronous on `stream`; allocates nothing.
 * Errors: RTS_E_UNSUPPORTED for plans built with conjugate=1, RTS_E_INVALID,
 * RTS_E_HIP. */
rts_status rts_chi2_backward(rts_plan_t plan, const float *vis, const float *weights, const float *model,
                             const float *grid_resid, const double *grad_chi2, float *grad_vis,
                             float *grad_weights, float *grad_grid, void *stream);

/* One cadence step as a HIP graph: rts_plan_update(uvw_m, weights) followed by
 * rts_grid_degrid(vis, weights, grid_in -> model_out, grid_out, chi2_out) is
 * captured once (on a private stream, after the work already queued on `stream`)
 * and each rts_cadence_graph_launch replays both over whatever the same buffers
 * hold at launch time, e.g. the next cadence's uvw, weights and visibilities.
 * All buffers must stay allocated at the same addresses while the graph lives;
 * the capture contains no allocation, memset or host synchronisation.  The
 * work-list capacity limit of rts_plan_update applies (rts_plan_info.n_dropped).
 * The limits of rts_grid_degrid apply: matrix-core plans need model_out; plans
 * with conjugate copies return RTS_E_UNSUPPORTED. */
rts_status rts_cadence_graph_create(rts_graph_t *out, rts_plan_t plan, const double *uvw_m,
                                    const float *vis, const float *weights, const float *grid_in,
                                    float *model_out, float *grid_out, double *chi2_out, void *stream);
rts_status rts_cadence_graph_launch(rts_graph_t graph, void *stream);
rts_status rts_cadence_graph_destroy(rts_graph_t graph);   /* NULL is accepted */

/* Tile-size autotuner: builds a plan for every legal tile edge in {16, 32, 64},
 * times three cadence steps (rts_plan_update + rts_grid_degrid) of each on the
 * given inputs with HIP events, and returns the fastest in *best_tile.  The
 * choice is cached per (N, W, OS, C, B, T, conjugate, du) for the process; a
 * non-NULL ms_out forces a fresh measurement and receives up to `capacity`
 * per-candidate times (tiles_out the candidates, *n_tried their count).
 * Allocates scratch for the model and grid outputs; synchronises `stream`. */
rts_status rts_autotune_tile(const rts_params *params, const double *uvw_m, const double *freq_hz,
                             const float *weights, const float *vis, const float *grid_in,
                             void *stream, int32_t *best_tile, float *ms_out, int32_t *tiles_out,
                             int32_t capacity, int32_t *n_tried);

/* a1 exposed for exact testing: out[c][b][t] = {xs, ys, valid} (int32) where
 * (xs, ys) are the snapped oversampled coordinates floor((u f/(c du) + N/2) OS + 1/2)
 * of the +uv copy (0 when non-finite) and valid follows the rule above.
 * `out` is device memory of C*B*T*3 int32. */
rts_status rts_compute_coords(const rts_params *params, const double *uvw_m,
                              const double *freq_hz, const float *weights, int32_t *out,
                              void *stream);

/* mask[c][b][t] (device, C*B*T bytes) = 1 where the sample is valid for this plan
 * (w != 0 at plan time and every tap on the grid), else 0.  Used for the
 * gradients of the chi-squared step, whose residual is zero at invalid samples. */
rts_status rts_plan_valid_mask(rts_plan_t plan, uint8_t *mask, void *stream);

/* Dirty image of every channel's grid (the imaging step after gridding,
 * Section 3, timed in Table 3): image[c] = shift(IFFT2(shift(grid[c]))) / (khat(nu_y) khat(nu_x)),
 * the centred inverse 2-D FFT without 1/N^2 normalisation, divided by the
 * separable grid correction, khat the Fourier transform of the plan's
 * Kaiser-Bessel window and nu = (q - N/2) / N for pixel q (pixel N/2 is l = 0).
 * grid and image_out: complex64 [C][N][N] device buffers, 16-byte aligned,
 * caller-owned; they may be the same buffer (in place), which with N a multiple
 * of 4 saves one pass over the grids (the grid is transformed as it is and one
 * pass exchanges the quadrants while applying sign and correction; out of place a
 * sign pass copies the modulated grid into image_out first).  The first call builds
 * the plan's FFT plan (batched over channels) and correction table, which
 * allocates device memory and copies the table synchronously; later calls
 * allocate nothing and are asynchronous on `stream`.
 * Errors: RTS_E_INVALID (NULL or misaligned), RTS_E_NOMEM, RTS_E_HIP. */
rts_status rts_image(rts_plan_t plan, const float *grid, float *image_out, void *stream);

/* Polarisation conversion (the polarisation convertor stage, Section 3; timed in
 * Tables 3 and 4): for every pixel i of every channel c, S_i = A_i P_i, where P_i
 * holds the pixel's four observed polarisation products and A_i is a 4x4 complex
 * matrix supplied by a precomputation:
 *     S[c][r][i] = sum_{k<4} A[r*4 + k][i] * P[c][k][i].
 * Layouts (device memory, complex64 as interleaved float, caller-owned):
 *   A  [16][n_pix]     entry r*4+k of every pixel's matrix, one plane per entry;
 *                      channel c reads the planes starting a_chan_stride complex
 *                      elements after A's start times c (a_chan_stride = 0: one
 *                      set of matrices for all channels; else >= 16*n_pix)
 *   P  [C][4][n_pix]   observed products, one plane per polarisation
 *   S  [C][4][n_pix]   output; S may be the same buffer as P (in place), but must
 *                      not overlap it otherwise, nor overlap A
 * Pointers must be 8-byte aligned; with 16-byte alignment, an even n_pix and an
 * even a_chan_stride, two pixels are converted per thread with 16-byte accesses.
 * n_pix == 0 or n_chan == 0 is a no-op (pointers unchecked).  Asynchronous on
 * `stream`; allocates nothing.
 * Errors: RTS_E_INVALID (negative sizes, bad stride, NULL or misaligned
 * pointers), RTS_E_HIP. */
rts_status rts_polconvert(const float *A, const float *P, float *S, int64_t n_pix, int n_chan,
                          int64_t a_chan_stride, void *stream);

/* Streaming device copy of `bytes` bytes from src to dst (device memory, not
 * overlapping, both 16-byte aligned): each byte is read once and written once with
 * 16-byte vector accesses, the bulk access pattern of the tile kernels.  It is the
 * reference for the attainable HBM bandwidth that throughput figures are reported
 * beside (not part of the method).  bytes == 0 is a no-op.  Asynchronous on
 * `stream`; allocates nothing.
 * Errors: RTS_E_INVALID (negative size, NULL, misaligned or overlapping buffers),
 * RTS_E_HIP. */
rts_status rts_stream_copy(const void *src, void *dst, int64_t bytes, void *stream);

/* Per-visibility kernels (Section 3: the gridder's kernel is fixed by the
 * calibration of the two tiles of each visibility's baseline; Table 4 uses a
 * 24 x 24 kernel).  After this call rts_grid and rts_degrid of a matrix-core plan
 * (RTS_PREC_BF16X3 or RTS_PREC_FP32_MFMA) use,
 * for every sample of baseline b, the separable kernel of that baseline instead
 * of the shared Kaiser-Bessel window:
 *     grid[c][cy+t_v][cx+t_u] += w V tab[b][r_y][t_v] tab[b][r_x][t_u],
 * with tab a device FP32 array [B][OS][W] in the phase / tap layout of
 * rts_plan_get_table (same along u and v, the same for every channel; conjugate
 * copies use their baseline's table at their own phases).  The values are copied
 * into plan-owned padded tables (about 8*B*2*OS*(W+32) bytes, allocated on the
 * first call); tab may be freed once the stream has passed this call.  A NULL tab
 * frees them and restores the shared kernel.  rts_grid, rts_degrid,
 * rts_grid_degrid and cadence graphs of the plan all use them while set.  New
 * tables replace the old ones at the same address (a live cadence graph replays
 * with them); adding or removing tables while a cadence graph of the plan is
 * alive returns RTS_E_INVALID.
 * Errors: RTS_E_UNSUPPORTED (not a matrix-core plan), RTS_E_INVALID, RTS_E_NOMEM,
 * RTS_E_HIP. */
rts_status rts_plan_set_baseline_kernels(rts_plan_t plan, const float *tab, void *stream);

/* Copy the FP32 kernel table tab[p][j] = k(t_j - r_p/OS) (OS rows, W columns; rows
 * are phases r0..r0+OS-1, columns taps t0..t0+W-1 with r0 = -(OS/2), t0 = -(W-1)/2
 * for odd W and r0 = 0, t0 = -W/2+1 for even W) into host memory `tab`
 * of `capacity` floats. */
rts_status rts_plan_get_table(rts_plan_t plan, float *tab, int64_t capacity);

rts_status rts_plan_get_info(rts_plan_t plan, rts_plan_info *info);

/* Release the plan and its workspace (waits for the device). NULL is accepted.
 * RTS_E_INVALID (nothing released) while a cadence graph of the plan is alive. */
rts_status rts_plan_destroy(rts_plan_t plan);

/* Message of the last failed call on this thread ("" if none). */
const char *rts_last_error(void);

/* Library version string. */
const char *rts_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RTSGRID_H */
