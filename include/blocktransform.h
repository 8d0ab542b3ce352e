/*
 * blocktransform.h -- C ABI of the MI355X (gfx950) block-transform library.
 *
 * The operation.  J. Selva's non-iterative type-4/5 NFFT methods reduce every
 * regular-grid step to one operator: evaluate a filtered trigonometric
 * polynomial on a uniform grid.  With the kernel coefficients Lambda of
 * eq. (4) and the coefficient vector S of eq. (34), the polynomial of eq. (6)
 * read at t = u/N is
 *
 *     y_u = sum_{n<N} Lambda_n S_n exp(+j 2 pi n u / N),        u < N.
 *
 * Its coset u = M q is eq. (7): a filter multiply, a circular fold of the
 * length-N spectrum onto K bins and a length-K IDFT (the paper's P is K here,
 * its oversampling factor eta is M, so N = K*M is its R = eta*P).  Evaluating
 * all M cosets makes the map square; when no Lambda_n is zero it is inverted
 * by eq. (31) generalised from the damping filter exp(-2 pi n a) of eq. (8)
 * to any nonzero real filter:
 *
 *     S_n = (N Lambda_n)^{-1} sum_u y_u exp(-j 2 pi n u / N).
 *
 * The adjoint is the Hermitian of the forward matrix (the same pairing that
 * relates the type-4 and type-5 systems, Sec. 6).  DFT signs and
 * normalisation follow eq. (0); the IDFT carries 1/P, as eq. (7) requires.
 *
 * Data layout.  A batch is `nblocks` blocks of N = K*M points.  Complex
 * arrays are complex64: interleaved (re, im) float32, block-major, natural
 * index order inside a block ([nblocks][N]).  Taps are float32: either one
 * shared vector [N] (tap_stride = 0) or one vector per block (tap_stride = N,
 * [nblocks][N]).
 *
 * Supported sizes.  K a power of two in [1, 1024]; M in [1, 16].  Other
 * values return TF_EUNSUPPORTED.  nblocks = 0 is a valid empty call.
 *
 * Ownership and ordering.  Every pointer passed to a transform call is a
 * device pointer owned by the caller, except the ragged layout arrays given to
 * transform_ragged_plan_create, which are host arrays copied by the library.
 * The library allocates only when a (K, M) schedule is first used on a device
 * (its twiddle table) and when a ragged plan is created; transform calls
 * themselves never allocate.  All transform calls are asynchronous on
 * `stream` (a hipStream_t; NULL means the default stream).  Inputs and
 * outputs must not overlap.
 *
 * Errors.  Arguments are validated on the host before any launch; no
 * exception crosses this interface.  Conditions found on the device (a zero
 * tap in an inverse) are reported through `status_dev`, and the affected
 * outputs then hold Inf/NaN by IEEE rules.
 */
#ifndef BLOCKTRANSFORM_H
#define BLOCKTRANSFORM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TF_OK = 0,
    TF_EINVAL = -1,         /* bad argument: null/overlapping/misaligned pointer, negative size */
    TF_EUNSUPPORTED = -2,   /* K or M outside the supported set, or unsupported compute mode */
    TF_ESINGULAR = -3,      /* reserved for host-detected singular filters */
    TF_EHIP = -4,           /* a HIP runtime call failed (launch, copy, allocation) */
    TF_EWORKSPACE = -5      /* workspace missing or smaller than transform_workspace_size() */
} tf_status;

typedef enum {
    TF_FP32 = 0,            /* fused single-pass kernel, FP32 arithmetic */
    TF_PLAIN_FP32 = 3,      /* unfused comparison path: one kernel per stage, HBM between stages */
    TF_SPLIT_BF16 = 1,      /* stage DFTs as BF16 hi+lo MFMA GEMMs, FP32 accumulation */
    TF_SPLIT_FP16 = 2       /* stage DFTs as scaled FP16 hi+lo MFMA GEMMs, FP32 accumulation */
} tf_compute;
/* The split modes serve transform_forward and transform_adjoint (without
   taps_bar) for K in {256, 1024}, M in [1, 16]; measured relative L2 against an
   FP64 reference is about 6e-6 (BF16) and 2e-7 (FP16), bounded by
   3 * 2^-2p * (4 + 2 sqrt(sqrt(K))) with p = 8 (BF16) or 11 (FP16). */

/*
 * transform_forward -- y = T(S): y_u = sum_n Lambda_n S_n e^{+j 2 pi n u/N}
 * (eq. (6) on the grid u/N; eq. (7) is its u = M q coset).
 *   coeffs   in : S, complex64 [nblocks][N]
 *   taps     in : Lambda, float32 [N] (tap_stride 0) or [nblocks][N] (tap_stride N)
 *   samples  out: y, complex64 [nblocks][N]
 *   compute     : a tf_compute value
 *   workspace   : device scratch of at least transform_workspace_size(...) bytes
 *                 (0 bytes for TF_FP32; NULL allowed when 0 is required)
 */
int transform_forward(const void *coeffs, const float *taps, void *samples,
                      int64_t nblocks, int32_t K, int32_t M, int64_t tap_stride,
                      int32_t compute, void *workspace, size_t workspace_bytes,
                      void *stream);

/*
 * transform_inverse -- S = T^{-1}(y): S_n = (N Lambda_n)^{-1} sum_u y_u e^{-j 2 pi n u/N}
 * (eq. (31) with the damping filter of eq. (8) replaced by any nonzero filter).
 *   samples    in : y, complex64 [nblocks][N]
 *   coeffs     out: S, complex64 [nblocks][N]
 *   status_dev out: nullable device int32; the kernel stores 1 into it when it
 *                   meets a zero tap (it never clears it: zero it first)
 */
int transform_inverse(const void *samples, const float *taps, void *coeffs,
                      int64_t nblocks, int32_t K, int32_t M, int64_t tap_stride,
                      int32_t compute, int32_t *status_dev,
                      void *workspace, size_t workspace_bytes, void *stream);

/*
 * transform_adjoint -- the Hermitian of the forward, and the filter gradient.
 *   W_n = sum_u ybar_u e^{-j 2 pi n u/N};   Sbar_n = Lambda_n W_n;
 *   Lambdabar_n = Re(conj(S_n) W_n), summed over blocks when taps are shared.
 *   samples_bar in : ybar, complex64 [nblocks][N]
 *   coeffs      in : S, complex64 [nblocks][N]; nullable unless taps_bar is given
 *   coeffs_bar  out: Sbar, complex64 [nblocks][N]
 *   taps_bar    out: nullable; float32 [N] (shared) or [nblocks][N] (per block).
 *                    The shared reduction is deterministic (fixed summation
 *                    order) and needs the workspace.
 */
int transform_adjoint(const void *samples_bar, const float *taps, const void *coeffs,
                      void *coeffs_bar, float *taps_bar,
                      int64_t nblocks, int32_t K, int32_t M, int64_t tap_stride,
                      int32_t compute, void *workspace, size_t workspace_bytes,
                      void *stream);

/*
 * transform_adjoint_noalloc -- transform_adjoint (FP32) for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same arguments and results as transform_adjoint with compute = TF_FP32, but
 * no workspace: the shared tap gradient's partial rows live in a device array of the
 * library (transform_noalloc_scratch_bytes(), 16 MiB, one copy per GPU, held until the
 * process ends); the launch grid is capped so that they fit, which can change the order of
 * the partial sums against transform_adjoint (results differ by rounding only).  Calls no
 * allocating routine.  All calls on one GPU share that array: calls that overlap in time on
 * one GPU (two streams, two threads) race and must not be issued; calls on one stream are
 * ordered and safe.  Errors as transform_adjoint; TF_EWORKSPACE if even a one-workgroup
 * grid's partial rows would not fit (cannot happen for N <= 16384).
 */
int transform_adjoint_noalloc(const void *samples_bar, const float *taps, const void *coeffs,
                              void *coeffs_bar, float *taps_bar,
                              int64_t nblocks, int32_t K, int32_t M, int64_t tap_stride,
                              void *stream);

/* Size in bytes of the device array transform_adjoint_noalloc uses (per GPU). */
size_t transform_noalloc_scratch_bytes(void);

/*
 * transform_inverse_adjoint -- the Hermitian of the inverse, and its filter gradient
 * (what autograd needs behind transform_inverse).
 *   ybar_u = sum_n e^{+j 2 pi n u/N} gbar_n / (N Lambda_n);
 *   Lambdabar_n = -Re(conj(gbar_n) Shat_n) / Lambda_n, summed over blocks when shared,
 *   where Shat is the inverse's output.
 *   coeffs_bar  in : gbar, complex64 [nblocks][N]
 *   coeffs      in : Shat, nullable unless taps_bar is given
 *   samples_bar out: ybar, complex64 [nblocks][N]
 */
int transform_inverse_adjoint(const void *coeffs_bar, const float *taps, const void *coeffs,
                              void *samples_bar, float *taps_bar,
                              int64_t nblocks, int32_t K, int32_t M, int64_t tap_stride,
                              int32_t compute, void *workspace, size_t workspace_bytes,
                              void *stream);

/*
 * transform_decimated -- eq. (7): the polynomial of eq. (6) read at the K regular
 * points q/K only (filter, circular fold of the N = K M spectrum onto K bins,
 * K-point IDFT):  out_q = sum_{n<N} Lambda_n S_n e^{+j 2 pi n q / K},  q < K.
 *   coeffs  in : S, complex64 [nblocks][N]
 *   taps    in : float32 [N] (tap_stride 0) or [nblocks][N] (tap_stride N)
 *   samples out: complex64 [nblocks][K]
 * K a power of two in [16, 1024], M in [1, 4096].
 */
int transform_decimated(const void *coeffs, const float *taps, void *samples, int64_t nblocks,
                        int32_t K, int32_t M, int64_t tap_stride, void *stream);

/*
 * transform_decimated_adjoint -- Hermitian of transform_decimated:
 *   Sbar_n = Lambda_n sum_{q<K} ybar_q e^{-j 2 pi n q / K},  n < N.
 *   samples_bar in : complex64 [nblocks][K]
 *   coeffs_bar  out: complex64 [nblocks][N]
 */
int transform_decimated_adjoint(const void *samples_bar, const float *taps, void *coeffs_bar,
                                int64_t nblocks, int32_t K, int32_t M, int64_t tap_stride,
                                void *stream);

/* Bytes of device workspace a call with these arguments needs (0 when none).
   `with_tapbar` is 1 when the call computes taps_bar. */
size_t transform_workspace_size(int64_t nblocks, int32_t K, int32_t M, int64_t tap_stride,
                                int32_t compute, int32_t with_tapbar);

/* Build the (K, M) schedule's tables on the current device ahead of time
   (for instance before stream capture).  Synchronous. */
int transform_prepare(int32_t K, int32_t M, int32_t compute);

/* Human-readable name of a tf_status value (static storage). */
const char *transform_status_string(int status);

/* Text of the last HIP error seen by the calling thread (after TF_EHIP). */
const char *transform_last_error(void);

/* ---------------------------------------------------------------- schedules
 * A (K, M) pair can run under several compiled schedules (radix plan, threads
 * per block, blocks per workgroup).  The autotuner times them and records the
 * winner; the choices persist as a small JSON file.
 */

/* Number of compiled fused schedules for (K, M); 0 when unsupported. */
int transform_schedule_count(int32_t K, int32_t M);

/* Describe schedule `idx` of (K, M) into `buf` (JSON object text). */
int transform_schedule_describe(int32_t K, int32_t M, int32_t idx, char *buf, size_t buflen);

/* Select schedule `idx` for (K, M) on all devices (idx -1: back to the default)
   and the grid cap in workgroups (0: automatic). */
int transform_schedule_select(int32_t K, int32_t M, int32_t idx, int32_t grid_cap);

/* The schedule index (0 = default) and grid cap currently selected for (K, M). */
int transform_schedule_selected(int32_t K, int32_t M, int32_t *idx, int32_t *grid_cap);

/* Load / save the selections as JSON ({"K,M": [idx, grid_cap], ...}). */
int transform_load_schedule(const char *json_path);
int transform_save_schedule(const char *json_path);

/* ---------------------------------------------------------------- ragged batches
 * A ragged batch is nblocks blocks with their own (K_b, M_b); block b's
 * points live at complex offset x_off[b] of the flat arrays and its taps at
 * float offset tap_off[b] (per-block taps only).  The plan groups the blocks
 * by class into tiles, cuts them into work items sorted by cost, and one
 * launch runs one workgroup per item in that order.  Supported classes:
 * K_b in {64, 128, 256, 512, 1024} and M_b in {3, 5, 7, 9, 15} (25 compiled
 * classes); any other (K_b, M_b) makes plan creation return TF_EUNSUPPORTED.
 * Concurrency: a launch keeps no state in the plan's device memory, so
 * executions of one plan may run on several streams at once.  The plan's HIP
 * graphs are cached per direction and pointer set under the plan's lock.
 */
typedef struct tf_ragged_plan_s *tf_ragged_plan;

/* Build a plan on the current device from host arrays of length nblocks.
   `total_points` is the length of the flat complex arrays.  Allocates. */
int transform_ragged_plan_create(const int32_t *K, const int32_t *M, const int64_t *x_off,
                                 const int64_t *tap_off, int64_t nblocks, int64_t total_points,
                                 tf_ragged_plan *plan);
/* The same with an explicit work-item size: each item is up to `chunk_tiles`
   tiles (a tile fills one workgroup with blocks of one class); 0 picks four.
   Larger items pipeline more tiles through each workgroup, smaller ones balance
   better; the autotuner chooses.  Whatever the value, no item carries more than a
   quarter of one workgroup slot's share of the batch's points (slots: the
   device's CUs times two), so classes of large blocks may get fewer tiles per
   item, down to one. */
int transform_ragged_plan_create_ex(const int32_t *K, const int32_t *M, const int64_t *x_off,
                                    const int64_t *tap_off, int64_t nblocks, int64_t total_points,
                                    int32_t chunk_tiles, tf_ragged_plan *plan);
int transform_ragged_plan_destroy(tf_ragged_plan plan);

/* direction: 0 forward, 1 inverse, 2 adjoint (taps_bar per block, nullable; needs aux = S).
   `use_graph` replays a HIP graph captured on first use for these pointers. */
int transform_ragged_execute(tf_ragged_plan plan, int32_t direction, const void *in,
                             const float *taps, void *out, const void *aux, float *taps_bar,
                             int32_t *status_dev, int32_t use_graph, void *stream);

/* Autotuned choice of the ragged kernel's tile pipelining, per class (K, M) and body:
   body 0 is the input side (forward), 1 the output side (inverse, adjoint), 2 the adjoint with
   the per-block tap gradient.  prefetch = 0 makes the class's tiles fetch their pass-0 operands
   when they start; 1 (or -1, the compiled default) fetches each tile's operands while the
   previous tile of the work item runs its LDS passes, where that body is compiled with the
   prefetch (it is where it fits the kernel's register budget).  Both forms compute the same
   arithmetic; as they are compiled separately, results may differ in rounding (relative
   differences near 1e-7).  The choice is process-wide and taken by plans created
   afterwards.  Returns TF_EINVAL for a body or prefetch value out of range, TF_EUNSUPPORTED for
   a (K, M) outside the 25 classes or prefetch = 1 where the body has no prefetching form (the
   (1024, 15) half-block body has none; `transform_ragged_prefetch_selected` reports which). */
int transform_ragged_prefetch_select(int32_t K, int32_t M, int32_t body, int32_t prefetch);
/* The prefetch setting in effect for (K, M, body): *prefetch = 0 or 1. */
int transform_ragged_prefetch_selected(int32_t K, int32_t M, int32_t body, int32_t *prefetch);

/* ---------------------------------------------------------------------------
 * Non-iterative type-5 and type-4 NFFT methods (Secs. "Computation of the
 * type-5 NFFT" / "Computation of the type-4 NFFT"), batched over independent
 * problems of P instants each.  The non-uniform steps are exact type-1/type-2
 * sums; the regular-grid steps are the block transforms above (the decimated
 * eq. (7) operator with the taps of eq. (41) for eq. (28); the inverse with the
 * damping filter of eq. (8) for eq. (43) and eq. (31); the forward with it for
 * eq. (37)).  Shared arguments:
 *   t        in : instants, float64 [nblocks][P], read modulo 1 (the sums are
 *                 1-periodic in t); converted to 64-bit fixed point on the device
 *   nblocks     : problems in the batch, 0..65535 (0: nothing is launched)
 *   P           : instants per problem, a power of two in [16, 1024]
 *   eta         : oversampling of eq. (28), R = eta P, 1..16
 *   a           : damping of the shifted grid q/P + ja, > 0; eq. (49) ties it
 *                 to the truncation ratio mu = e^{-2 pi (eta P - 1) a}/(eta P - 1)
 *   workspace   : device scratch of nufft_workspace_size(nblocks, P, eta)
 *                 bytes, 256-byte aligned, owned by the caller
 * Arithmetic: exact fixed-point phases; the exact non-uniform sums in FP64
 * (FP64 exponential tables, products on the FP64 matrix cores); FP32 everywhere
 * else.  All work is asynchronous on
 * `stream`; errors are reported before any launch (TF_EINVAL for bad pointers,
 * overlaps or a, TF_EUNSUPPORTED for P/eta outside the ranges, TF_EWORKSPACE).
 * --------------------------------------------------------------------------- */
size_t nufft_workspace_size(int64_t nblocks, int32_t P, int32_t eta);

/* options of nufft_solve */
enum {
    NUFFT_REFINE = 1,    /* the refined method of Sec. 5 (eq. (44)-(46)) */
    NUFFT_GRIDDING = 2   /* non-uniform sums by the gridding NFFTs below instead of exact
                            sums: needs 2 eta P <= 16384 (a block-transform size) */
};
size_t nufft_workspace_size_ex(int64_t nblocks, int32_t P, int32_t eta, int32_t flags);

/* type 4 or 5 with options; the four entry points below are its fixed-option forms */
int nufft_solve(int32_t type, int32_t flags, const double *t, const void *in, void *out,
                int64_t nblocks, int32_t P, int32_t eta, double a, void *workspace,
                size_t workspace_bytes, void *stream);

/* The same in two steps, for several inputs on the same instants.  nufft_setup
   computes the part of both methods that depends on the instants only (the
   filters of eq. (8) and eq. (41), the kernel samples of eq. (28)-(29), the
   Lagrange coefficients of eq. (43) and the derivative samples of eq. (16)) into
   the workspace; nufft_apply then runs type 4 or 5 (with NUFFT_REFINE if asked)
   from that workspace, as often as wanted, and leaves the setup intact.  The
   caller guarantees that the workspace holds a setup of the same t, nblocks, P,
   eta and a; NUFFT_GRIDDING may differ between the two calls if the workspace is
   large enough for the gridding flag of each.  In nufft_setup the flags select
   only how its sums are evaluated.  Errors as for nufft_solve. */
int nufft_setup(int32_t flags, const double *t, int64_t nblocks, int32_t P, int32_t eta, double a,
                void *workspace, size_t workspace_bytes, void *stream);
int nufft_apply(int32_t type, int32_t flags, const double *t, const void *in, void *out, int64_t nblocks,
                int32_t P, int32_t eta, double a, void *workspace, size_t workspace_bytes, void *stream);

/* type 5 (inverse of eq. (34), the system eq. (48)): coefficients S_p, p < P,
   from samples s(t_q).  samples in: complex64 [nblocks][P]; coeffs out: same. */
int nufft_type5(const double *t, const void *samples, void *coeffs, int64_t nblocks, int32_t P,
                int32_t eta, double a, void *workspace, size_t workspace_bytes, void *stream);

/* type 4 (inverse of eq. (32), the system eq. (47) with p = 0..P-1): amplitudes
   a_q from the spectrum A(r), r < P.  spectrum in / amplitudes out: complex64
   [nblocks][P]. */
int nufft_type4(const double *t, const void *spectrum, void *amplitudes, int64_t nblocks, int32_t P,
                int32_t eta, double a, void *workspace, size_t workspace_bytes, void *stream);

/* the refined methods of Sec. 5 (eq. (44)-(46)): one pass of the method, the
   residual of the system computed with the exact type-2 (type 5) or type-1
   (type 4) sum, a second pass on the residual, subtracted.  The relative error
   of one pass, eps, becomes about eps^2 (down to the FP32 floor).  Same
   arguments as above; the input and output must not overlap. */
int nufft_type5_refined(const double *t, const void *samples, void *coeffs, int64_t nblocks, int32_t P,
                        int32_t eta, double a, void *workspace, size_t workspace_bytes, void *stream);
int nufft_type4_refined(const double *t, const void *spectrum, void *amplitudes, int64_t nblocks,
                        int32_t P, int32_t eta, double a, void *workspace, size_t workspace_bytes,
                        void *stream);

/* Gridding NFFTs (the type-1 NFFT of Sec. 2 as one gridding operation and one FFT at
   oversampling 2; the type-2 as a weighting, an inverse FFT and a short interpolation).
   Window: the periodised Gaussian exp(-x^2/(4 tau)) of Dutt-Rokhlin / Greengard-Lee,
   tau = ln(1e7)/(2 pi^2 n^2), 16 grid points per instant, fine grid n = 2 band, relative
   accuracy about 1e-7 (FP32).  The band (R for type 1, P for type 2) must be even, >= 16, with
   2 band <= 16384 a block-transform size (K M, K a power of two <= 1024, M <= 16).
   Same array layouts as nudft_type1 / nudft_type2; workspace of nfft_workspace_size
   bytes, 256-byte aligned. */
size_t nfft_workspace_size(int64_t nblocks, int32_t band);
int nfft_type1(const double *t, const void *amp, void *out, int64_t nblocks, int32_t Q, int32_t R,
               void *workspace, size_t workspace_bytes, void *stream);
int nfft_type2(const double *t, const void *coeffs, void *out, int64_t nblocks, int32_t P, int32_t Q,
               void *workspace, size_t workspace_bytes, void *stream);

/* exact type-1 sum, eq. (32): out[b][r] = sum_{q<Q} amp[b][q] e^{-j 2 pi r t[b][q]}, r < R.
   t: float64 [nblocks][Q]; amp: complex64 [nblocks][Q], NULL for unit amplitudes;
   out: complex64 [nblocks][R].  Q in [1, 65536], R in [1, 65536]. */
int nudft_type1(const double *t, const void *amp, void *out, int64_t nblocks, int32_t Q, int32_t R,
                void *stream);

/* exact type-2 sum, eq. (34): out[b][q] = sum_{p<P} coeffs[b][p] e^{+j 2 pi p t[b][q]}, q < Q.
   t: float64 [nblocks][Q]; coeffs: complex64 [nblocks][P]; out: complex64 [nblocks][Q].
   P in [1, 65536], Q in [1, 65536]. */
int nudft_type2(const double *t, const void *coeffs, void *out, int64_t nblocks, int32_t P, int32_t Q,
                void *stream);

#ifdef __cplusplus
}
#endif

#endif /* BLOCKTRANSFORM_H */
