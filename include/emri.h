/*
 * emri.h -- C ABI of the MI355X (gfx950) library for the semi-coherent
 * EMRI track search (arXiv 2510.20891).
 *
 * The library builds a PSD-normalised SFT power spectrogram (or the whitened
 * complex SFTs) from a time series, builds an SVD basis of frequency tracks,
 * and scores very large batches of basis-coefficient vectors against the
 * spectrogram: every track is rebuilt at every segment midpoint, the power in
 * its nearest frequency bin is looked up, the lookups are summed over
 * segments and the best tracks are kept (top-k).  Beside this nearest-bin
 * statistic it evaluates the 201-bin linear-chirp statistic
 * (score_tracks_chirp), a multi-harmonic statistic (score_tracks_harmonics),
 * many independent streams in one launch (score_batched_*), and the
 * population search over coefficients (search_*).
 *
 * Conventions shared by every call
 *   - Plain C types only.  Pointers documented as "device" point to GPU memory
 *     (for instance a PyTorch tensor's data_ptr()); "host" pointers to CPU memory.
 *   - Every buffer, including the scoring workspace, is allocated by the caller.
 *     The library never allocates device memory.  Device calls only enqueue
 *     work on `hip_stream` (a hipStream_t; NULL is the default stream) and
 *     return without synchronising, except the set-up calls score_batched_plan,
 *     search_seed and search_plan, which wait for their own table copies.
 *     Outputs are valid once the caller has synchronised that stream.
 *   - Every call returns an emri_status.  Arguments are validated before any HIP
 *     call; on failure nothing is enqueued and emri_last_error() describes why.
 *     Nothing is thrown or aborted across the boundary.
 *   - Device pointers must be 16-byte aligned.
 */
#ifndef EMRI_H
#define EMRI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EMRI_OK = 0,
  EMRI_EINVAL = -1,       /* a NULL required pointer, a size or value out of range */
  EMRI_ERANGE = -2,       /* a size product overflows                             */
  EMRI_ENOMEM = -3,       /* the workspace passed is smaller than required        */
  EMRI_EDEVICE = -4,      /* a HIP call or kernel launch failed                   */
  EMRI_EUNSUPPORTED = -5  /* a valid request the library does not implement      */
} emri_status;

typedef enum {
  EMRI_F32 = 0,           /* normalised power, FP32                                          */
  EMRI_F16 = 1,           /* normalised power, FP16                                          */
  EMRI_C32 = 2            /* whitened complex SFT, (re, im) FP32 pairs (linear-chirp statistic) */
} emri_pdtype;

/* A normalised-power spectrogram in device memory, owned by the caller.
 * Row alpha (segment alpha) holds P[alpha, b] for bins b = 0..n_bins-1 at
 * data[alpha * row_pitch + b]; elements n_bins..row_pitch-1 of a row are padding
 * that scoring never reads as power.  row_pitch is a multiple of 8 elements and
 * at least n_bins; data is 16-byte aligned. */
typedef struct {
  void *data;
  int32_t n_seg;          /* number of segments (rows)                                  */
  int32_t n_bins;         /* bins per row = n_sft/2 + 1                                  */
  int32_t row_pitch;      /* elements between consecutive rows                           */
  int32_t dtype;          /* emri_pdtype                                                 */
  double t_sft;           /* segment duration T_SFT in seconds; bin b is at b / T_SFT Hz */
} emri_power;

/* Arithmetic of the track contraction sum_k c_k U[alpha, k] T_SFT. */
typedef enum {
  EMRI_PLAIN = 0,         /* FP64 fused multiply-adds on the vector units                     */
  EMRI_MIXED = 1          /* BF16 matrix cores on 3-piece split operands, FP32 accumulation;  */
                          /* f0 T_SFT and the rounding to a bin stay FP64 (1 <= K <= 16)      */
} emri_precision;

/* Options for score_tracks; a NULL pointer selects the defaults. */
typedef struct {
  int32_t k_min;          /* lowest bin that contributes (default 0)                      */
  int32_t k_max;          /* highest bin that contributes; < 0 means n_bins - 1 (default) */
  int32_t precision;      /* emri_precision (default EMRI_PLAIN)                          */
  int32_t reserved[4];    /* must be zero                                                 */
  int32_t rescore_top;    /* EMRI_MIXED with top_k > 0: 1 re-scores the leading candidates */
                          /* with FP64 positions before the top-k (see score_tracks)       */
} score_opts;

/*
 * build_sfts -- normalised SFT power of a real time series.
 *
 * Sec. II B cuts the data into SFT segments of duration T_SFT (bin width
 * 1/T_SFT) and weights every bin by the inverse PSD (Eq. (7)); Sec. II F takes
 * the PSD as known.  Segment alpha is samples [alpha*n_sft, (alpha+1)*n_sft) of
 * x (n_seg = n_samples / n_sft; trailing samples are dropped).  Each segment is
 * multiplied by the periodic Hann window w_n = sin^2(pi n / n_sft), transformed
 * with a real DFT (FP64, computed on the GPU), and
 *     P[alpha, b] = |X_b|^2 / ((3 n_sft / 8) * psd[b] / (2 dt)),
 * where 3 n_sft / 8 = sum_n w_n^2.  Bins whose psd is non-positive or not finite
 * get P = 0.  With this normalisation noise-only power is Exp(1) distributed.
 *
 *   x          device FP64[n_samples]
 *   dt         sample spacing in seconds (finite, > 0)
 *   n_sft      samples per segment: even, >= 4, n_sft/2 with no prime factor
 *              above 7, and n_sft <= 20480 (EMRI_EUNSUPPORTED otherwise)
 *   psd        device FP64[n_sft/2 + 1], one-sided PSD at f_b = b / (n_sft dt)
 *   out        caller-owned spectrogram: out->data (device, n_seg*row_pitch
 *              elements), out->row_pitch and out->dtype are read; n_seg, n_bins
 *              and t_sft are written.  Padding elements are written as 0.
 *              FP16 storage rounds to nearest (values above the FP16 range
 *              become +inf).  With dtype EMRI_C32 an element is the whitened
 *              complex SFT Z[alpha, b] = X_b / sqrt((3 n_sft / 8) psd[b] / (2 dt))
 *              as two FP32 values (re, im), so |Z|^2 is the power above; bins
 *              with a non-positive or non-finite psd hold 0.  Only the
 *              linear-chirp statistic (score_tracks_chirp) reads C32 data.
 */
int build_sfts(const double *x, int64_t n_samples, double dt, int32_t n_sft,
               const double *psd, emri_power *out, void *hip_stream);

/*
 * build_basis -- centred SVD basis of training frequency tracks (host, FP64,
 * synchronous; no GPU involved).
 *
 * Sec. II C factorises the matrix of training tracks with the SVD (Eq. (9)) and
 * writes a track as a combination of leading singular vectors (Eq. (10)); the
 * coefficient prior is uniform within symmetric 3-sigma quantiles.  Here
 *   f0[alpha]    = mean over training tracks (the basis is centred),
 *   U[:, k]      = k-th right singular vector of the centred matrix, k < K,
 *                  sign chosen so that its largest-magnitude entry is positive
 *                  (lowest alpha on a tie),
 *   sv[k]        = k-th singular value (descending),
 *   box_lo/hi[k] = 0.135 % / 99.865 % quantiles (linear interpolation) of the
 *                  training projections (F - f0) U[:, k].
 * A track is then f(t_alpha) = f0[alpha] + sum_k c_k U[alpha, k].
 *
 *   tracks   host FP64[n_train * n_seg], row-major (one training track per row), Hz
 *   K        0 <= K <= min(n_train, n_seg)
 *   f0       host FP64[n_seg];  U host FP64[n_seg * K] row-major (U[alpha*K + k])
 *   sv, box_lo, box_hi   host FP64[K]
 */
int build_basis(const double *tracks, int64_t n_train, int32_t n_seg, int32_t K,
                double *f0, double *U, double *sv, double *box_lo, double *box_hi);

/*
 * score_tracks_workspace_size -- bytes of device workspace score_tracks needs
 * for these sizes (stat == NULL needs room for the statistic as well).
 */
int score_tracks_workspace_size(const emri_power *power, int32_t K, int64_t n_tmpl,
                                int32_t top_k, int32_t stat_in_workspace, size_t *bytes);

/*
 * score_tracks -- nearest-bin semi-coherent statistic and top-k of a batch.
 *
 * Eq. (6) sums the per-segment statistic over segments; for a template that
 * occupies one bin per segment (the zero-bandwidth limit of the linear-chirp
 * template of Sec. II B) the per-segment term is the normalised power in that
 * bin.  With tracks rebuilt by the matrix product of Eq. (10):
 *     x[j, alpha] = (f0[alpha] + sum_k c[j, k] U[alpha, k]) * T_SFT   (FP64)
 *     b[j, alpha] = rint(x[j, alpha])          (round half to even)
 *     S[j]        = sum over alpha with k_min <= b <= k_max of P[alpha, b]
 * Non-finite positions contribute nothing.  Positions are evaluated in FP64
 * (f0 T_SFT + sum_k c_k (U T_SFT) with fused multiply-adds), so chosen bins
 * agree with any FP64 evaluation except within ~1e-12 bin of a half-integer.
 * The statistic is accumulated in FP32 over runs of 8 segments and in FP64
 * across runs (relative error below 1e-6), and stored as FP32.  Sec. II D
 * keeps the best candidates of a batch: the top-k is ordered by decreasing S
 * and then increasing template index; NaN statistics rank below every number.
 *
 *   power      spectrogram (FP32 or FP16), device
 *   f0         device FP64[n_seg]; U device FP64[n_seg * K] row-major
 *   K          0..32
 *   coeffs     device FP32[n_tmpl * K] row-major (one template per row)
 *   n_tmpl     0 <= n_tmpl <= 2^31 - 1
 *   top_k      0..4096
 *   stat       device FP32[n_tmpl] or NULL (then the workspace holds it)
 *   topk_val   device FP32[top_k]; topk_idx device INT64[top_k]; entries past
 *              n_tmpl are (-inf, -1).  Both may be NULL when top_k == 0.
 *   bins       device INT32[n_tmpl * n_seg] or NULL: if given, the chosen bin of
 *              every (template, segment), -1 where it does not contribute.
 *   n_near_tie device INT64[1] or NULL: if given, set to the number of
 *              (template, segment) positions within 1e-6 bin of a half-integer.
 *   (bins and n_near_tie select a slower validation kernel.)
 *   opts       NULL or bin range, precision and re-scoring options
 *
 * With precision EMRI_MIXED the positions are FP32 sums (see emri_precision):
 * a position within the FP32 error (~1e-4 bin at 10^3 bins) of a half-integer
 * can take the neighbouring bin, so a small share of templates carries one
 * moved bin.  Above K = 8 templates whose coefficients 8..15 carry little of
 * the contraction (at most 2^-9 and 2^-17 of its bound for groups 8..11 and
 * 12..15) skip the smallest split products of those groups, which moves a
 * position by at most 2.5 * 2^-24 of the contraction bound (the FP32
 * accumulation of the full products already rounds 24 times by up to 2^-24
 * of its partial sums); the others are scored with every product.  Either
 * way a statistic depends on its own template only, and the batched form
 * (score_batched_run) returns the same statistics bit for bit.
 * With rescore_top = 1 (and top_k > 0) the call takes the
 * kc = min(n_tmpl, max(4 top_k, 64), 4096) best templates of the mixed
 * statistic, evaluates each again exactly as the plain path does (its FP64
 * statistic bit for bit, written into stat), and returns the best top_k of
 * those kc; the plain path ignores rescore_top.
 *
 *   workspace  device, at least score_tracks_workspace_size() bytes, 256-byte
 *              aligned; its contents on entry are irrelevant.
 */
int score_tracks(const emri_power *power, const double *f0, const double *U, int32_t K,
                 const float *coeffs, int64_t n_tmpl, int32_t top_k,
                 float *stat, float *topk_val, int64_t *topk_idx,
                 int32_t *bins, int64_t *n_near_tie, const score_opts *opts,
                 void *workspace, size_t workspace_bytes, void *hip_stream);

/*
 * score_tracks_noalloc -- score_tracks for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, arithmetic, kernels and results as
 * score_tracks, without the workspace: the library keeps a fixed scratch of
 * score_tracks_noalloc_limit() bytes (4 MiB) per GPU in static device memory,
 * held until the process ends, and this call allocates nothing.  A request
 * whose workspace (score_tracks_workspace_size with stat_in_workspace = (stat
 * == NULL)) exceeds that limit fails with EMRI_ENOMEM before any HIP call;
 * one-year shapes with any top_k need about 0.3 MB when stat is given.
 * Every call on a GPU uses that GPU's one scratch: calls that overlap on one
 * GPU (concurrent streams, or threads) race and must be serialised by the
 * caller.  Each call re-initialises what it reads from the scratch.
 */
int score_tracks_noalloc(const emri_power *power, const double *f0, const double *U, int32_t K,
                         const float *coeffs, int64_t n_tmpl, int32_t top_k,
                         float *stat, float *topk_val, int64_t *topk_idx,
                         int32_t *bins, int64_t *n_near_tie, const score_opts *opts, void *hip_stream);

/* Bytes of the static scratch score_tracks_noalloc uses on each GPU. */
size_t score_tracks_noalloc_limit(void);

/*
 * score_tracks_harmonics -- the multi-harmonic statistic (Sec. IV proposes
 * adding harmonics at a cost proportional to their number).  Harmonic h
 * follows the searched track scaled by the fixed frequency ratio ratios[h]
 * (host FP64[n_harm], finite, in (0, 1024]; e.g. 1, 1/2, 3/2 for the m = 2,
 * 1, 3 harmonics of a circular orbit), and every harmonic's nearest-bin power
 * is summed:
 *     S[j] = sum_alpha sum_h P[alpha, rint(ratios[h] x[j, alpha])]
 * over bins inside [k_min, k_max], with x as in score_tracks (FP64) and the
 * scaled position rounded half to even as one fused operation (bins agree
 * with rint of the FP64 product except within ~1e-12 bin of a half-integer).
 * 1 <= n_harm <= 4 and 1 <= K <= 16 (EMRI_EUNSUPPORTED otherwise); the
 * precision option must be EMRI_PLAIN.  Other arguments, the workspace
 * (score_tracks_workspace_size) and the top-k are as in score_tracks; each
 * harmonic costs one more gather per template and segment.
 */
int score_tracks_harmonics(const emri_power *power, const double *f0, const double *U, int32_t K,
                           const float *coeffs, int64_t n_tmpl, int32_t n_harm, const double *ratios,
                           int32_t top_k, float *stat, float *topk_val, int64_t *topk_idx,
                           const score_opts *opts, void *workspace, size_t workspace_bytes, void *hip_stream);

/*
 * score_tracks_chirp -- the linear-chirp statistic of Sec. II B (Eqs. (4)-(7))
 * over 2P + 1 bins, the paper's own statistic (score_tracks is its one-bin,
 * zero-bandwidth limit).  Per template and segment alpha, with the track
 * f[alpha] = f0[alpha] + sum_k c_k U[alpha, k] (FP64), fdot and fddot its
 * second-order finite differences over the segment grid (central inside,
 * one-sided fdot at the ends, the neighbour's fddot at the ends), k0 =
 * rint(f T) inside the row and fdot T^2 finite in FP32 (else the segment
 * contributes nothing) and, over the bins k = k0 - P..k0 + P inside the row,
 *     H_k      = R(f T - k, fdot T^2) (up to a factor common to all k),
 *     R(d, b)  = int_{-1/2}^{1/2} cos^2(pi u) exp(2 pi i d u + i pi b u^2) du
 *                (the SFT of the Hann-windowed unit linear chirp, Eqs. (4)-(5)),
 *     S_alpha  = |sum_k conj(Z_k) H_k / sqrt(psd_k)|^2 / sum_k |H_k|^2 / psd_k
 * ((max over phase of <d|h>)^2 / <h|h>, Eq. (6)-(7), without the constant
 * 3/4 = 2 sum w^2 / N, so that P = 0 gives the nearest-bin power), and
 *     S = sum over segments with |fddot| T^3 / 6 <= 1, f >= f_min and
 *         fdot >= fdot_min of S_alpha    (Sec. II B validity cut, Sec. II D cut-offs).
 * R is evaluated as the 256-point DFT of its Hann-windowed samples (relative
 * error below 4e-7 for |fdot T^2| <= 60), in FP32; sums over bins in FP32
 * per lane and FP64 across lanes, over segments in FP64; S stored FP32.
 *
 *   sfts     complex whitened SFTs from build_sfts with dtype EMRI_C32
 *            (n_seg <= 2048)
 *   psd      device FP64[n_bins]; bins with psd <= 0 or not finite take no part
 *   f0, U, K, coeffs, n_tmpl, top_k, stat, topk_val, topk_idx  as in score_tracks
 *   opts     NULL for P = 100, f_min = 10^-3.5 Hz, fdot_min = 1e-13 Hz/s;
 *            pass -INFINITY to disable a cut-off; 0 <= p_half <= 100
 *   workspace  score_tracks_chirp_workspace_size() bytes, 256-byte aligned
 */
typedef struct {
  int32_t p_half;            /* P: the window is 2P + 1 bins                    */
  int32_t pad;
  double f_min;              /* Hz: segments below contribute nothing           */
  double fdot_min;           /* Hz/s: segments below contribute nothing         */
  int32_t reserved[4];       /* must be zero                                    */
} chirp_opts;

int score_tracks_chirp_workspace_size(const emri_power *sfts, int32_t K, int64_t n_tmpl, int32_t top_k,
                                      int32_t stat_in_workspace, size_t *bytes);
int score_tracks_chirp(const emri_power *sfts, const double *psd, const double *f0, const double *U, int32_t K,
                       const float *coeffs, int64_t n_tmpl, int32_t top_k, float *stat, float *topk_val,
                       int64_t *topk_idx, const chirp_opts *opts, void *workspace, size_t workspace_bytes,
                       void *hip_stream);

/*
 * Batched form: many scoring problems in one persistent launch.
 *
 * A problem is one batch of coefficient vectors scored against one
 * spectrogram exactly as score_tracks does (several problems may share a
 * spectrogram, e.g. many requests against a few resident data streams).  All
 * problems of a batch share K and the power storage type; their spectrogram
 * shapes, segment counts, template counts, bin ranges and top_k may differ.
 * Each template's statistic is summed in the same order as in score_tracks, so
 * every result is bit-for-bit the one a standalone score_tracks call gives.
 *
 * score_batched_plan validates the problems, splits them into work items of
 * one or two tiles of templates ordered by decreasing cost (workgroups claim
 * them through a counter), and writes the launch tables into the workspace
 * with host-to-device copies on hip_stream.  Unlike every other call it then
 * waits for hip_stream to drain (the copies read host memory the call owns),
 * so it must not be called while a graph is being captured on hip_stream.
 * score_batched_run only launches kernels
 * that read those tables, so it may be captured into a HIP graph and replayed;
 * a replay re-reads the problems' current device inputs.  The plan stays valid
 * while the workspace and every problem buffer stay allocated.
 */
typedef struct {
  emri_power power;          /* spectrogram of this problem                        */
  const double *f0;          /* device FP64[n_seg]                                  */
  const double *U;           /* device FP64[n_seg * K]                              */
  const float *coeffs;       /* device FP32[n_tmpl * K]                             */
  int64_t n_tmpl;            /* 0 .. 2^31 - 1                                       */
  int32_t top_k;             /* 0 .. 4096                                           */
  int32_t k_min, k_max;      /* bin range; k_max < 0 means n_bins - 1               */
  int32_t reserved;          /* must be zero                                        */
  float *stat;               /* device FP32[n_tmpl], or NULL (kept in the workspace)*/
  float *topk_val;           /* device FP32[top_k] (may be NULL if top_k == 0)      */
  int64_t *topk_idx;         /* device INT64[top_k]                                 */
} emri_problem;

typedef struct {
  int32_t rows_per_step;       /* spectrogram rows staged per step: 0 = as many as fit, or 1, 2, 4 */
  int32_t templates_per_lane;  /* 0 = default; otherwise a value score_batched_tile_options lists  */
  int32_t precision;           /* emri_precision (EMRI_MIXED stages 4 rows per step)               */
  int32_t reserved[5];         /* must be zero                                                     */
} batch_opts;

typedef struct {
  int64_t opaque[24];          /* filled by score_batched_plan; caller-owned, not interpreted */
} emri_batch_plan;

/* Bytes of workspace a batch needs (256-byte aligned workspace required). */
int score_batched_workspace_size(const emri_problem *problems, int32_t n_problems, int32_t K, size_t *bytes);

/* Templates-per-lane values compiled for K (written to out[0..*n_out)); the
 * first is the default.  Used by autotuners. */
int score_batched_tile_options(int32_t K, int32_t *out, int32_t *n_out);

int score_batched_plan(const emri_problem *problems, int32_t n_problems, int32_t K, const batch_opts *opts,
                       void *workspace, size_t workspace_bytes, emri_batch_plan *plan, void *hip_stream);

int score_batched_run(const emri_batch_plan *plan, void *hip_stream);

/*
 * Population search (Sec. II D): the walkers of a search are coefficient
 * vectors in the prior box, seeded from uniform draws and improved by the
 * track-space differential-evolution step of Eq. (11).  A chain is one
 * population scored against one spectrogram and basis; many chains advance
 * together (one batched scoring launch per generation), e.g. one per
 * observed duration of the progressive search, whose basis is the one-year
 * basis shifted by a whole number of segments (f0 and U pointing
 * n_seg_full - n_seg rows in, so the track ends at the chosen plunge).
 * Tracks are projected back onto a chain's basis rows with their
 * pseudo-inverse, which the set-up calls compute on the host (FP64, singular
 * values below 1e-15 of the largest dropped).  Random numbers (candidate
 * draws, initial frequencies, partners, weights) are inputs.
 */
typedef struct {
  emri_power power;          /* the chain's spectrogram rows (n_seg >= 1)                   */
  const double *f0;          /* device FP64[n_seg]                                          */
  const double *U;           /* device FP64[n_seg * K], finite                              */
  const double *box_lo;      /* device FP64[K]: prior box of the coefficients, inclusive   */
  const double *box_hi;      /* device FP64[K]                                              */
  float *coeffs;             /* device FP32[n_walkers * K]: the walkers, updated in place  */
  float *stat;               /* device FP32[n_walkers]: their statistics, updated in place */
  int32_t n_walkers;         /* >= 3                                                        */
  int32_t k_min, k_max;      /* contributing bin range; k_max < 0 means n_bins - 1         */
  int32_t reserved;          /* must be zero                                                */
} emri_chain;

typedef struct {
  int64_t opaque[40];        /* filled by search_plan; caller-owned, not interpreted        */
} emri_search_plan;

/*
 * search_seed -- Sec. II D's initial population, for every chain: candidate j
 * of chain c is draws[(c * n_draw + j) * K ...] (device FP32, uniform in the
 * box); its track f = f0 + U c is moved by one constant so that its first
 * segment is at f_init[c * n_draw + j] Hz (device FP64), projected back onto
 * the basis with its pseudo-inverse (FP32), scored, and the chain's n_walkers best by (-S, index)
 * (n_walkers <= min(n_draw, 4096)) become its walkers, with their statistics.
 * opts selects the scoring precision and tile (as score_batched_plan).
 * A set-up call: like score_batched_plan it waits for its table copies.
 */
int search_seed_workspace_size(const emri_chain *chains, int32_t n_chains, int32_t K, int32_t n_draw, size_t *bytes);
int search_seed(const emri_chain *chains, int32_t n_chains, int32_t K, const float *draws, const double *f_init,
                int32_t n_draw, const batch_opts *opts, void *workspace, size_t workspace_bytes, void *hip_stream);

/*
 * search_plan / search_generation -- Eq. (11).  search_plan (a set-up call
 * that waits for its table copies) writes the chains' tables and the trials'
 * scoring plan into the workspace.  search_generation then, for every walker
 * i of every chain (walkers of chain c numbered from the sum of the earlier
 * chains' n_walkers in the concatenated draws):
 *     f_trial = f_i + F[i] (f_r1[i] - f_r2[i])        (tracks in FP64)
 *     c_trial = pinv(U) (f_trial - f0), stored FP32
 * scores every trial (one batched launch), and replaces walker i by its trial
 * if every c_trial[k] lies in [box_lo[k], box_hi[k]] and the trial's
 * statistic is strictly higher.  r1, r2: device INT32 partner indices within
 * the chain (walkers whose r1, r2, i are not three different walkers in range
 * keep their vector); F: device FP64 weights; accepted: device INT32 (1 if
 * replaced) or NULL.  search_generation only launches kernels: it may be
 * captured into a HIP graph.  The plan stays valid while the workspace and
 * the chains' buffers stay allocated.
 */
int search_workspace_size(const emri_chain *chains, int32_t n_chains, int32_t K, size_t *bytes);
int search_plan(const emri_chain *chains, int32_t n_chains, int32_t K, const batch_opts *opts,
                void *workspace, size_t workspace_bytes, emri_search_plan *plan, void *hip_stream);
int search_generation(const emri_search_plan *plan, const int32_t *r1, const int32_t *r2, const double *F,
                      int32_t *accepted, void *hip_stream);

/*
 * search_generations -- n_gen >= 0 generations of Eq. (11), each exactly as
 * search_generation (same trials, statistics and acceptance, bit for bit):
 * generation g takes r1, r2 and F from row g of device arrays of n_gen x
 * (total walkers of the plan) entries.  Two generations at a time run as one
 * launch each, reading one copy of the population and writing the other (the
 * second copy lives in the plan's workspace), so that every trial sees the
 * population of the previous generation; an odd last generation runs as
 * search_generation does.  When the call's work is done the population is in
 * the chains' coeffs and stat.  Launches only: it may be captured into a HIP
 * graph.
 */
int search_generations(const emri_search_plan *plan, int32_t n_gen, const int32_t *r1, const int32_t *r2,
                       const double *F, void *hip_stream);

/*
 * search_best -- per chain, the best walker by (-S, index) (NaN ranks last):
 * best_stat FP32[n_chains], best_idx INT32[n_chains]; and, if best_norm is
 * given (FP64[n_chains]), its statistic normalised by the chain's noise-only
 * mean and standard deviation (device FP64[n_chains] each), the per-duration
 * normalisation of Sec. II D.
 */
int search_best(const emri_search_plan *plan, const double *noise_mean, const double *noise_std,
                float *best_stat, int32_t *best_idx, double *best_norm, void *hip_stream);

/*
 * search_noise_moments -- Sec. II D normalises each duration's statistic by
 * its mean and standard deviation under noise-only data: over n_real >= 2
 * noise-only searches, best[r * n_chains + c] (device FP32) is chain c's best
 * statistic in realisation r; mean and sd (device FP64[n_chains]) receive the
 * mean and the sample standard deviation (denominator n_real - 1).
 */
int search_noise_moments(const float *best, int32_t n_real, int32_t n_chains, double *mean, double *sd,
                         void *hip_stream);

/* Human-readable name of a status code (static storage). */
const char *emri_status_string(int status);

/* Detail of the last failing call on this thread ("" if none; thread-local storage). */
const char *emri_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EMRI_H */
