/*
 * sincos.h -- C ABI of libmi355_sincos.so: the branch-free single-precision
 * sine-cosine pair of M. H. Mendenhall, "A Fast, Vectorizable Algorithm for
 * Producing Single-Precision Sine-Cosine Pairs" (2004), on AMD Instinct MI355X
 * (gfx950).
 *
 * The pair (s, c) of an angle x (radians) is computed in binary32 by the
 * paper's steps: x is scaled by 1/(2 pi) and reduced modulo 1 by rounding to
 * the nearest integer (ties to even) and subtracting (Sec. II); odd and even
 * series give sin and cos of a quarter of the reduced turn (Sec. II, the
 * polynomials of the chosen method); two angle doublings use the stable form
 * of eq. (1); the pair is finally multiplied by a magnitude factor taken after
 * the first doubling (Sec. II, magnitude correction; Fig. 1).
 *
 * Conventions for every entry point:
 *  - Array pointers are DEVICE pointers owned by the caller.  The library never
 *    frees them and keeps no reference after the call returns (plans keep the
 *    pointers they were created with; see below).  Host tables passed in
 *    (segment lists, lengths) are copied before the call returns.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *    it asynchronously; no call synchronizes the stream.  A fault inside a
 *    kernel is reported by the caller's next synchronization, not here.
 *  - Arguments are checked on the host before anything is enqueued; on error
 *    nothing is enqueued and the call returns a negative status, with a
 *    message available from sincos_last_error() on the same thread.
 *  - n == 0 is a valid no-op.  Arrays must be 4-byte aligned; any 4-byte
 *    alignment works (a float4 body is used when x, s and c share their
 *    offset modulo 16 bytes, scalar elements otherwise).
 *  - In place: x == s or x == c is allowed (each element is read before its
 *    outputs are written).  s == c, or any other overlap between x, s and c,
 *    is rejected with SINCOS_EOVERLAP.
 *  - Special values: +-Inf and NaN give (NaN, NaN).  |x| >= 2^23 * 2 pi
 *    (~5.27e7) reduces to a zero angle and gives (0, 1) exactly: this is what
 *    the binary32 sequence computes, not a correct sine.
 */
#ifndef MI355_SINCOS_H
#define MI355_SINCOS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#ifndef SINCOS_API
#define SINCOS_API __attribute__((visibility("default")))
#endif

typedef enum {
    SINCOS_OK = 0,
    SINCOS_EINVAL = -1,   /* bad size, null or misaligned pointer, bad option */
    SINCOS_EOVERLAP = -2, /* forbidden aliasing between inputs and outputs    */
    SINCOS_ENOMEM = -3,   /* a library-owned device or host buffer failed     */
    SINCOS_EHIP = -4,     /* the HIP runtime returned an error                */
    SINCOS_ENODEV = -5,   /* no usable gfx950 device is current               */
    SINCOS_ECANCELED = -6, /* request dropped because its server shut down    */
    SINCOS_EBUDGET = -7   /* request larger than the server's whole budget   */
} sincos_status_t;

/* Arithmetic of the multiply-adds.
 * FUSED: each multiply-add of the paper's AltiVec form is one fused operation
 *        (one rounding), as AltiVec's vector multiply-add is.  Default.
 * SPLIT: every product and every sum is rounded on its own (the same
 *        expression tree, built with floating-point contraction off).
 * CONTRACT: the SPLIT expression tree compiled with contraction allowed; the
 *        compiler may fuse any product into a following sum.  Each component
 *        is within 2^-20 + pi * ulp(fl(x / (2 pi))) (absolute) of SPLIT: the
 *        second term is the rounding of the scaled angle, which a fused
 *        reduction skips.
 * FUSED and SPLIT are bit-exact against the CPU oracle of the same mode. */
typedef enum {
    SINCOS_ARITH_FUSED = 0,
    SINCOS_ARITH_SPLIT = 1,
    SINCOS_ARITH_CONTRACT = 2
} sincos_arith_t;

/* Series and magnitude fix (Sec. II).
 * NORMALIZED: the first method: least-squares series of sin and cos, factor
 *             2 - s^2 - c^2.  Default.
 * ARCTAN:     the second method: series fit to the angle only, factor
 *             1 / (s^2 + c^2) by correctly rounded division. */
typedef enum {
    SINCOS_METHOD_NORMALIZED = 0,
    SINCOS_METHOD_ARCTAN = 1
} sincos_method_t;

/* Launch shape (0 in a field = the form's default: the built-in one below,
 * or what sincos_set_tuning installed).
 * block:  threads per workgroup, a multiple of 64 in [64, 1024]; built-in 64
 *         for the plain form, 256 for the ragged form.
 * unroll: float4 per thread per loop trip (1, 2, 4 or 8); built-in 1.
 * grid:   workgroups; built-in 0 = one per tile, covering the array once
 *         (grid-stride beyond 2^30 workgroups or 2^32 work-items); for the
 *         ragged form one per unit of work, and a smaller grid makes the
 *         launch persistent.
 * lds:    bytes of LDS each workgroup reserves at launch (up to 65536),
 *         which caps how many workgroups a CU holds at once (a CU has
 *         160 KiB); -1 = reserve none.  Built-in: 7168 for the plain form
 *         (at most 22 resident 64-thread workgroups per CU, which keeps
 *         fewer DRAM rows open at once: measured 1-2 % faster on MI355X),
 *         none for the ragged form.  Used by the plain and ragged forms and
 *         the memory probes; other forms ignore it.                         */
typedef struct {
    int32_t block;
    int32_t unroll;
    int32_t grid;
    int32_t lds;
} sincos_launch_t;

/* ---------------------------------------------------------------------- */
/* Plain form: s[i], c[i] = pair(x[i]) for 0 <= i < n (SoA outputs).
 * Default arithmetic FUSED, method NORMALIZED, default launch shape.      */
SINCOS_API int sincos_f32(const float *x, float *s, float *c, int64_t n, void *stream);

/* Same with explicit arithmetic, method and launch shape (launch may be
 * NULL).                                                                  */
SINCOS_API int sincos_f32_ex(const float *x, float *s, float *c, int64_t n, int32_t arith, int32_t method,
                  const sincos_launch_t *launch, void *stream);

/* Interleaved outputs: the same pairs (FUSED, NORMALIZED) written to one
 * array.
 *   layout 0: complex64 e^{ix}: out[2i] = cos x_i, out[2i+1] = sin x_i
 *             (out holds 2 n floats);
 *   layout 1: the phase blocks of the paper's sample implementation: for each
 *             4 consecutive elements, 4 sines then 4 cosines (out holds
 *             8 ceil(n/4) floats; a final partial block leaves its unused slots
 *             untouched).
 * x and out 16-byte aligned, no overlap between them.                     */
SINCOS_API int sincos_f32_interleaved(const float *x, float *out, int64_t n, int32_t layout,
                                      void *stream);

/* ---------------------------------------------------------------------- */
/* Ragged form: `count` independent arrays in ONE kernel launch.
 * segs[j] = {x_j, s_j, c_j} (device pointers), lens[j] >= 0 its length.
 * Both tables are host memory, read before the call returns.  Each segment
 * obeys the plain form's aliasing rules; in addition no output may overlap
 * any other segment's input or output (inputs may be shared).
 * Up to 64 non-empty segments the descriptor table is passed in the kernel
 * arguments; larger tables are staged through library-owned pinned and
 * device buffers (a small ring guarded by events).  Either way the call
 * must not be made while `stream` is being captured into a graph: use a
 * plan for that.                                                          */
typedef struct {
    const float *x;
    float *s;
    float *c;
} sincos_seg_t;

SINCOS_API int sincos_f32_ragged(const sincos_seg_t *segs, const int64_t *lens, int32_t count, void *stream);

SINCOS_API int sincos_f32_ragged_ex(const sincos_seg_t *segs, const int64_t *lens, int32_t count,
                         int32_t arith, int32_t method, const sincos_launch_t *launch,
                         void *stream);

/* Ragged plan: the segment table is validated and copied to device memory
 * once (synchronously, on the current device); launching it is then a
 * single kernel launch with no host work and no allocation, safe to capture
 * in a HIP graph.  The plan keeps the segment pointers: the caller keeps the
 * arrays alive and may change their contents (not their addresses) between
 * launches.  A plan is used from one thread at a time.                    */
typedef struct sincos_ragged_plan sincos_ragged_plan_t;

SINCOS_API int sincos_ragged_plan_create(const sincos_seg_t *segs, const int64_t *lens, int32_t count,
                              int32_t arith, int32_t method, const sincos_launch_t *launch,
                              sincos_ragged_plan_t **out_plan);
/* Enqueue the plan's kernel on `stream`.  Both launch calls need the
 * plan's device to be current (EINVAL otherwise).                         */
SINCOS_API int sincos_ragged_plan_launch(const sincos_ragged_plan_t *plan, void *stream);
/* Enqueue the plan as a HIP graph (built by stream capture of the kernel on
 * the first call and instantiated once; later calls replay it).          */
SINCOS_API int sincos_ragged_plan_graph_launch(sincos_ragged_plan_t *plan, void *stream);
/* Shape the plan resolved to (any field may be NULL). */
SINCOS_API int sincos_ragged_plan_info(const sincos_ragged_plan_t *plan, int32_t *block, int32_t *unroll,
                            int32_t *grid, int64_t *units, int64_t *elements);
/* Free the plan's device table and graph.  Waits for nothing: the caller
 * makes sure no launch of the plan is still running.                      */
SINCOS_API int sincos_ragged_plan_destroy(sincos_ragged_plan_t *plan);

/* ---------------------------------------------------------------------- */
/* Adjoint of the pair (d sin/dx = cos, d cos/dx = -sin, the analytic
 * derivative evaluated with the approximated pair):
 *     gx[i] = gs[i] * c[i] - gc[i] * s[i]
 * each product and the difference rounded once in binary32.  gs or gc may
 * be NULL (treated as zero; both NULL writes +0).  gx may alias gs or gc
 * exactly; no other overlap with gx is allowed.                           */
SINCOS_API int sincos_f32_backward(const float *s, const float *c, const float *gs, const float *gc,
                        float *gx, int64_t n, void *stream);

/* ---------------------------------------------------------------------- */
/* Sinusoid model for least-squares fitting (the smooth-derivative use the
 * paper motivates in Sec. II):  y(t_i) = sum_k A_k sin(w_k t_i + phi_k).
 * In binary32: theta_ik = fma(w_k, t_i, phi_k); y_i accumulates
 * fma(A_k, s_ik, y_i) over k = 0..K-1 in order, starting from +0.  Uses
 * FUSED arithmetic and the NORMALIZED method for the pair.
 * t, y: [N] device arrays; A, w, phi: [K] device arrays; all 4-byte
 * aligned.  K >= 0.  y may be t exactly; any other overlap of y with t, A,
 * w or phi is EOVERLAP.                                                   */
SINCOS_API int sinusoid_f32_forward(const float *t, int64_t N, const float *A, const float *w,
                         const float *phi, int32_t K, float *y, void *stream);

/* The forward model fused with the residual and the loss of a least-squares
 * fit (Sec. II's use of the smooth pair):  r_i = y_i - y_obs_i in binary32,
 * with y_i exactly as sinusoid_f32_forward computes it, written to r; and
 * loss[0] = 1/2 sum_i r_i^2, summed in a fixed order (per lane with fma in
 * sample order, a 256-way tree per workgroup, then a tree over the
 * workgroups), so the result is deterministic.
 * t, y_obs, r: [N] device arrays; r may be t or y_obs exactly (no other
 * overlap).  loss: one device float (written also when N == 0, as +0).
 * workspace: device scratch of at least
 * sinusoid_f32_residual_workspace_bytes(N) bytes (one float per workgroup,
 * 4 ceil(N / 2048) bytes up to 4 MiB), owned by the caller.  r, loss and
 * the workspace's used bytes overlap neither each other nor t, y_obs, A, w,
 * phi (EOVERLAP), apart from the exact in-place r; all 4-byte aligned.    */
SINCOS_API int64_t sinusoid_f32_residual_workspace_bytes(int64_t N);
SINCOS_API int sinusoid_f32_residual(const float *t, const float *y_obs, int64_t N, const float *A,
                                     const float *w, const float *phi, int32_t K, float *r,
                                     float *loss, void *workspace, int64_t workspace_bytes,
                                     void *stream);

/* Gradients of a loss L with dL/dy_i = g_i:
 *     gA_k   = sum_i g_i s_ik
 *     gphi_k = A_k sum_i g_i c_ik
 *     gw_k   = A_k sum_i g_i c_ik t_i
 * (for L = 1/2 sum (y_i - y_obs_i)^2, g = y - y_obs).  Partial sums are taken
 * in binary32 per block of samples and combined in a fixed order, so the
 * result is deterministic.  gA, gw, gphi: [K] device outputs.  workspace:
 * device scratch of at least sinusoid_f32_backward_workspace_bytes(N, K)
 * bytes (3 * 64 ceil(K/64) ceil(N/2048) floats: one partial per 2048
 * samples and frequency), owned by the caller.  gA, gw, gphi and the
 * workspace's used bytes overlap neither each other nor t, g, A, w, phi
 * (EOVERLAP); all arrays 4-byte aligned.  EINVAL if N > 2^31 * 2048.      */
SINCOS_API int64_t sinusoid_f32_backward_workspace_bytes(int64_t N, int32_t K);
SINCOS_API int sinusoid_f32_backward(const float *t, const float *g, int64_t N, const float *A,
                          const float *w, const float *phi, int32_t K, float *gA, float *gw,
                          float *gphi, void *workspace, int64_t workspace_bytes, void *stream);

/* One step of the least-squares fit in one pass: with y_i as
 * sinusoid_f32_forward computes it and r_i = y_i - y_obs_i,
 *     loss[0] = 1/2 sum_i r_i^2,
 *     gA, gw, gphi = the gradients sinusoid_f32_backward gives for g = r
 * (the same bits as sinusoid_f32_residual followed by sinusoid_f32_backward;
 * the loss is summed in another fixed order, so its last bits may differ).
 * The residual stays on chip.  workspace: device scratch of at least
 * sinusoid_f32_fit_step_workspace_bytes(N, K) bytes ((3 * 64 ceil(K/64) + 1)
 * ceil(N/2048) floats), owned by the caller.  loss, gA, gw, gphi and the
 * workspace overlap neither each other nor t, y_obs, A, w, phi; all arrays
 * 4-byte aligned.  N == 0 gives loss 0 and zero gradients.                 */
SINCOS_API int64_t sinusoid_f32_fit_step_workspace_bytes(int64_t N, int32_t K);
SINCOS_API int sinusoid_f32_fit_step(const float *t, const float *y_obs, int64_t N, const float *A,
                                     const float *w, const float *phi, int32_t K, float *loss,
                                     float *gA, float *gw, float *gphi, void *workspace,
                                     int64_t workspace_bytes, void *stream);

/* sinusoid_f32_fit_step without a workspace argument, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, checks,
 * results and bits as sinusoid_f32_fit_step; the partials go to a static
 * device array of SINCOS_FIT_SCRATCH_BYTES that the library holds on each
 * GPU it runs on until the process ends (its address is looked up on the
 * first call per device, with that device current).  Nothing is allocated:
 * no hipMalloc, hipFree or allocating library call.  EINVAL when
 * sinusoid_f32_fit_step_workspace_bytes(N, K) exceeds
 * SINCOS_FIT_SCRATCH_BYTES (at K <= 64: N above 22,253,568 samples).
 * Every call writes all the scratch it reads before reading it, so nothing
 * needs clearing; but all calls on one GPU share the one array, so calls
 * that overlap in time on that GPU (other streams, other threads) race and
 * may return wrong results: serialize them.                               */
#define SINCOS_FIT_SCRATCH_BYTES (8 << 20)
SINCOS_API int sinusoid_f32_fit_step_noalloc(const float *t, const float *y_obs, int64_t N,
                                             const float *A, const float *w, const float *phi,
                                             int32_t K, float *loss, float *gA, float *gw,
                                             float *gphi, void *stream);

/* ---------------------------------------------------------------------- */
/* Huygens' principle point-source sum (the application named in Sec. IV):
 * the complex field at P screen points (xo_i, yo_i, L) from S point sources
 * in the plane z = 0,
 *     U_i = sum_j (a_j / r_ij) exp(i (k (r_ij - L) + phi_j)),
 * r_ij the distance, obliquity factor 1, the path difference r - L formed
 * as rho^2 / (r + L) (rho the lateral distance).  In binary32, each
 * operation rounded: dx, dy by subtraction, rho2 = fma(dx, dx, dy*dy),
 * r = sqrt(rho2 + fl(L*L)) correctly rounded, e = r + L, x = r*e; while x is
 * a normal binary32 both quotients come from one correctly rounded
 * reciprocal g = 1/x: d = rho2*(r*g), w = a_j*(e*g); otherwise d = rho2/e,
 * w = a_j/r (correctly rounded divisions).  theta = fma(k, d, phi_j), the
 * pair of theta (FUSED, NORMALIZED), re = fma(w, c, re), im = fma(w, s, im).
 * The sources are summed in 4 contiguous blocks of ceil(S/4), each in
 * source order from +0, and the block sums are added in block order.
 * xo, yo, re, im: [P] device arrays; src: [S][4] = (x, y, a, phi), device,
 * 16-byte aligned.  0 < L < 1e18 (else EINVAL).  Outputs may not overlap
 * any input.                                                              */
SINCOS_API int huygens_f32(const float *xo, const float *yo, int64_t P, const float *src,
                           int32_t S, float k, float L, float *re, float *im, void *stream);

/* Measurement helper: the Huygens term's own ceiling.  Exactly huygens_f32
 * over the 8 sources of src8 ([8][4] = (x, y, a, phi), device, 16-byte
 * aligned) repeated `reps` times (S = 8 * reps, sources in table order
 * within each repetition): the same kernel code as huygens_f32 with the
 * source index wrapped into the 8-entry table, which stays in the scalar
 * cache, i.e. the term's arithmetic with (almost) no source traffic.  Same
 * argument rules as huygens_f32; reps outside [0, 2^28) is EINVAL.        */
SINCOS_API int huygens_term_ceiling_f32(const float *xo, const float *yo, int64_t P,
                                        const float *src8, int32_t reps, float k, float L,
                                        float *re, float *im, void *stream);

/* ---------------------------------------------------------------------- */
/* Measurement helper: the same memory traffic as the plain form (read 4 B,
 * write 8 B per element, float4 body, same launch shape) with no
 * arithmetic: s[i] = x[i], c[i] = x[i].  Gives the measured bandwidth
 * ceiling for the plain kernel.                                           */
SINCOS_API int sincos_copy_ceiling_f32(const float *x, float *s, float *c, int64_t n,
                            const sincos_launch_t *launch, void *stream);

/* Measurement helper: memory-traffic probes for the plain form's roofline.
 * Each uses the plain kernel's buffer instructions with no arithmetic, over
 * n elements (n >= 0, a multiple of 4; arrays 16-byte aligned, pairwise
 * disjoint):
 *   SINCOS_PROBE_READ        reads x (4 B per element); writes at most
 *                            s[0], and only for inputs whose bits fold to a
 *                            fixed unlikely word (the store keeps the loads).
 *   SINCOS_PROBE_WRITE       writes s and c (8 B per element); x unused.
 *   SINCOS_PROBE_WRITE1      writes s only (4 B per element); x, c unused.
 *   SINCOS_PROBE_COPY        s = c = x in the plain kernel's schedule: one
 *                            tile of block * unroll float4 per workgroup,
 *                            s and c stored row by row (with the default
 *                            policy, what sincos_copy_ceiling_f32 does).
 *   SINCOS_PROBE_COPY_BATCH  s = c = x; a workgroup loads all `unroll` rows
 *                            of its tile, then stores every row of s, then
 *                            every row of c.
 *   SINCOS_PROBE_COPY_SPLIT  s = c = x; two-wave workgroups (block 128) over
 *                            64-float4 tiles: both waves load the tile, wave
 *                            0 stores s and wave 1 stores c.
 *   SINCOS_PROBE_COPY_LDS    s = c = x; two-wave workgroups over 128-float4
 *                            tiles read once into LDS: wave 0 stores the
 *                            tile to s, wave 1 to c.
 *   SINCOS_PROBE_COPY_XCD    s = c = x in the plain schedule with unroll 1,
 *                            the tiles dealt to the 8 XCDs in runs of
 *                            launch->grid consecutive tiles (1 = the plain
 *                            order; 0 = a contiguous eighth per XCD).
 * policy: -1 = the plain kernel's (loads non-temporal, stores sc1); for
 * READ, WRITE, WRITE1 and COPY also the cache-policy bits of the stores (of
 * the loads for READ): 0, 1 (sc0), 2 (nt), 16 (sc1), 17 (sc0|sc1) or 18
 * (nt|sc1).  launch: as for sincos_f32_ex (NULL = the plain form's
 * default, including its LDS reservation); the split and LDS probes
 * always use 128 threads.  EINVAL for an
 * unknown probe or policy or bad sizes, EOVERLAP for overlapping arrays.  */
enum {
    SINCOS_PROBE_READ = 0,
    SINCOS_PROBE_WRITE = 1,
    SINCOS_PROBE_WRITE1 = 2,
    SINCOS_PROBE_COPY = 3,
    SINCOS_PROBE_COPY_BATCH = 4,
    SINCOS_PROBE_COPY_SPLIT = 5,
    SINCOS_PROBE_COPY_LDS = 6,
    SINCOS_PROBE_COPY_XCD = 7
};
SINCOS_API int sincos_stream_probe_f32(int32_t probe, int32_t policy, const float *x, float *s,
                                       float *c, int64_t n, const sincos_launch_t *launch,
                                       void *stream);

/* Measurement helper: the VALU ceiling of the pair's instruction mix.  Lane i
 * runs 8 independent chains theta_r = x[i] + r (r = 0..7), adding 1 per step,
 * for `reps` steps; each step takes the pair (FUSED, NORMALIZED) of every
 * theta_r and adds its sine and cosine to two binary32 running sums (plain
 * adds, in step order).  out[i] = sum over r = 0..7, in order, of
 * (sines_r + cosines_r).  Register-only between one load and one store per
 * lane.  x and out: [n] device arrays, 4-byte aligned; out == x is allowed,
 * any other overlap is EOVERLAP.  n < 0 or reps < 0 is EINVAL.            */
SINCOS_API int sincos_pair_ceiling_f32(const float *x, float *out, int64_t n, int32_t reps,
                                       void *stream);

/* ---------------------------------------------------------------------- */
/* Ablations of Sec. II, for analysis and measurement.  Each element is
 * reduced as in step 1, then:
 *   sincos_f32_variant: the method's series (method 1 or 2) and one of
 *     LISTING   the method itself (the plain form's bits);
 *     NO_FIX    both doublings, no magnitude factor;
 *     TEXT_FIX  both doublings, then the text's factor (3 - s^2 - c^2)/2
 *               applied to the final pair (Sec. II, magnitude correction);
 *     EQ2       both doublings with the rejected eq. (2),
 *               cos 2a = 1 - 2 sin^2 a, and the method's factor.
 *   sincos_f32_doublings: the general form of the trade-off in Sec. II
 *     between series length and doublings: s1 = q (ss[0] + ss[1] q^2 + ...
 *     + ss[ns-1] q^(2 ns - 2)), c1 = 1 + q^2 (cc[0] + ... + cc[nc-1]
 *     q^(2 nc - 2)), by Horner in q^2, approximating sin and cos of
 *     2 pi q / 2^ndoub; then ndoub eq. (1) doublings.  With fix, the pair is
 *     scaled by 2 - s^2 - c^2 of the pair before the last doubling (for
 *     ndoub = 0, by (3 - s^2 - c^2)/2 of the series pair).  ndoub = 2, the
 *     first method's series and fix = 1 give the plain form's bits.
 * arith: FUSED or SPLIT (CONTRACT is EINVAL).  ss, cc: HOST arrays of ns and
 * nc binary32 coefficients (1 <= ns, nc <= 16), read before the call
 * returns; 0 <= ndoub <= 8.  x, s, c: [n] device arrays, 16-byte aligned;
 * the aliasing rules of the plain form.                                    */
typedef enum {
    SINCOS_VARIANT_LISTING = 0,
    SINCOS_VARIANT_NO_FIX = 1,
    SINCOS_VARIANT_TEXT_FIX = 2,
    SINCOS_VARIANT_EQ2 = 3
} sincos_variant_t;

SINCOS_API int sincos_f32_variant(const float *x, float *s, float *c, int64_t n, int32_t arith,
                                  int32_t method, int32_t variant, void *stream);
SINCOS_API int sincos_f32_doublings(const float *x, float *s, float *c, int64_t n, int32_t arith,
                                    int32_t ndoub, const float *ss, int32_t ns, const float *cc,
                                    int32_t nc, int32_t fix, void *stream);

/* ---------------------------------------------------------------------- */
/* Request server: continuous batching of sine-cosine requests of any size.
 *
 * A scheduler thread owns an output arena in device memory and up to
 * `max_inflight` streams.  Submitted requests queue in arrival order; a
 * request is admitted when its 12 n bytes fit in the HBM budget (4 n for the
 * input it pins, 8 n for its outputs) and an arena block is free.  Whenever
 * a stream is free, the admitted requests not yet launched go to the device
 * as ONE ragged launch (up to the batch caps), so requests that arrive while
 * others run join the next batch and batches overlap on the device.  With a
 * size split, requests of more than split_elems elements and smaller ones
 * never share a batch: the oldest waiting request decides the class, and
 * the batch takes the waiting requests of that class in arrival order, so a
 * small request never waits for a large one's batch to finish.  Batches of
 * one class run one after another on that class's stream, each at the rate
 * of the whole device, while the other class's stream overlaps them
 * (stream_per_slot = 1 instead lets every batch in flight share the device).
 * A completion carries the device addresses of the request's
 * outputs; they stay valid until the request is released (or at once with
 * auto_release).  Release returns the request's budget and arena block.
 * Each result is the same bits as a plain sincos_f32 call on the same input
 * (the kernels share the arithmetic).
 * Times are host steady-clock nanoseconds.  Inputs are device pointers owned
 * by the caller, which keeps them unchanged until the request completes.  */
typedef struct sincos_server sincos_server_t;

typedef struct {
    int64_t budget_bytes;       /* HBM admission budget (0 = 8 GiB)                     */
    int32_t max_inflight;       /* batches on the device at once (0 = 4, max 16)        */
    int32_t max_batch_requests; /* requests per batch (0 = 4096)                        */
    int64_t max_batch_elems;    /* elements per batch (0 = no cap)                      */
    int32_t arith;              /* sincos_arith_t                                        */
    int32_t method;             /* sincos_method_t                                       */
    int32_t mode;               /* 0 = continuous batching (one ragged launch per batch),
                                   1 = one plain launch per request (the baseline)       */
    int32_t executor;           /* 0 = the GPU; 1 = simulated (no device work, no device
                                   memory; completion after sim_* time; host tests)     */
    int64_t sim_batch_ns;       /* simulated: fixed time per batch                      */
    int64_t sim_elem_ps;        /* simulated: picoseconds per element                   */
    int32_t sim_fail_every;     /* simulated: every k-th batch fails (0 = never)        */
    int32_t auto_release;       /* 1 = free a request's outputs as soon as it completes */
    int64_t split_elems;        /* size split between batch classes (0 = 2^22 elements,
                                   -1 = no split: one class)                            */
    int32_t stream_per_slot;    /* 0 = the batches of one size class run in order on that
                                   class's stream, and the classes' streams overlap;
                                   1 = every batch in flight on a stream of its own, all
                                   overlapping (mode 1 always runs this way); else EINVAL */
    int32_t reserved;           /* set to 0                                              */
} sincos_server_config_t;

typedef struct {
    int64_t id;
    uint64_t tag;
    int32_t status;             /* SINCOS_OK, SINCOS_EHIP (batch failed), SINCOS_ECANCELED */
    int32_t batch_requests;     /* requests in the batch that carried it                 */
    const float *s;             /* device outputs, n each (NULL with auto_release)       */
    const float *c;
    int64_t n;
    int64_t t_submit_ns, t_admit_ns, t_launch_ns, t_complete_ns;
} sincos_completion_t;

typedef struct {
    int64_t submitted, admitted, completed, failed, batches;
    int64_t elements_completed;
    int64_t budget_in_use, budget_peak;
    int32_t inflight_peak;
    int32_t reserved;
} sincos_server_stats_t;

SINCOS_API int sincos_server_create(const sincos_server_config_t *cfg, sincos_server_t **out);
/* Queue a request of n >= 1 elements; *out_id receives its id.  Returns
 * SINCOS_EBUDGET if 12 n exceeds the whole budget.  x must already hold its
 * values for any stream (e.g. the producing stream was synchronized): the
 * server's streams are not ordered after the caller's.  Thread-safe.      */
SINCOS_API int sincos_server_submit(sincos_server_t *srv, const float *x, int64_t n, uint64_t tag,
                                    int64_t *out_id);
/* The same, for an input produced by work enqueued on `stream` (a
 * hipStream_t of the server's device; 0 = the null stream): an event is
 * recorded on `stream` now, and the batch that carries the request waits for
 * it on the device before reading x, so the caller need not synchronize.
 * The calling thread's current device must be the server's (else EINVAL).
 * x must stay allocated and unchanged until the request completes: a caller
 * that frees it (or lets an allocator reuse it) before then gets undefined
 * results.  A simulated server ignores `stream`.  Thread-safe.             */
SINCOS_API int sincos_server_submit_on(sincos_server_t *srv, const float *x, int64_t n,
                                       uint64_t tag, void *stream, int64_t *out_id);
/* Up to `max` completions (waits up to timeout_ns for the first one).     */
SINCOS_API int sincos_server_poll(sincos_server_t *srv, sincos_completion_t *out, int32_t max,
                                  int32_t *count, int64_t timeout_ns);
/* Give back a completed request's outputs and budget.                     */
SINCOS_API int sincos_server_release(sincos_server_t *srv, int64_t id);
SINCOS_API int sincos_server_stats(const sincos_server_t *srv, sincos_server_stats_t *out);
/* Submit request j at start + arrival_ns[j] from a generator thread, wait
 * for every completion and store it in out[j].  With auto_release off each
 * request is released once its completion is stored.  Request j carries tag
 * j and the replay consumes every completion it polls, so nothing else may
 * submit to or poll the server while a replay runs.                       */
SINCOS_API int sincos_server_replay(sincos_server_t *srv, const float *const *xs,
                                    const int64_t *ns, const int64_t *arrival_ns, int32_t count,
                                    sincos_completion_t *out);
/* Stop: pending (unadmitted) requests complete with SINCOS_ECANCELED,
 * batches on the device are waited for, then everything is freed.        */
SINCOS_API int sincos_server_destroy(sincos_server_t *srv);

/* ---------------------------------------------------------------------- */
/* Process-wide default launch shapes: the autotuner's hook.  The shape of a
 * call that passes no launch shape (and the fields it leaves 0) comes from
 * here: sincos_f32, sincos_f32_ex and sincos_copy_ceiling_f32 take "plain";
 * sincos_f32_ragged(_ex), ragged plans and the server's batches take
 * "ragged" (the server's one-launch-per-request mode takes "plain").
 * json: a JSON object {"plain": {...}, "ragged": {...}}, each holding any of
 *       the integer fields "block", "unroll", "grid", "lds" with the
 *       meanings and limits of sincos_launch_t.  Forms and fields left out
 *       get the built-in defaults (plain 64, 1, 0, 7168; ragged 256, 1, 0,
 *       0), so NULL or "{}" restores them.
 * Errors: EINVAL for text outside that form (unknown or repeated keys,
 * non-integers, whitespace or numbers JSON does not allow, trailing text)
 * or values out of range; the current shapes are then kept.
 * Thread-safe.  Takes effect for calls that start after it returns; plans
 * keep the shape they were created with.  No GPU is needed.              */
SINCOS_API int sincos_set_tuning(const char *json);

/* The shapes in effect, written as the JSON object sincos_set_tuning takes.
 * Writes at most cap - 1 characters and a terminating NUL into buf (buf may
 * be NULL when cap is 0); returns the full length of the text.            */
SINCOS_API int64_t sincos_get_tuning(char *buf, int64_t cap);

/* ---------------------------------------------------------------------- */
/* Message for the last non-OK status returned on this thread ("" if none). */
SINCOS_API const char *sincos_last_error(void);

/* Library version string. */
SINCOS_API const char *sincos_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MI355_SINCOS_H */
