/*
 * fastmap_hip.h - C ABI of the MI355X (gfx950) epipolar-adjustment library.
 *
 * Besides epipolar adjustment it holds the pose stages that feed it (further
 * below): global rotation averaging and its initialisation, the
 * relative-translation grid search, global translation averaging, and
 * focal-length refinement inside epipolar adjustment.
 *
 * The epipolar operations follow FastMap (arXiv 2505.04612), Sec. 3.3
 * "Epipolar Adjustment" and App. B.6:
 *
 *   pairs      P = {(i_n, j_n)}, i_n is the first image of pair n, j_n the second;
 *   matches    Q_n = {(x1_nm, x2_nm)}, normalised coordinates, homogeneous
 *              x~ = (u, v, 1); x1 lies in image i_n, x2 in image j_n;
 *   poses      world-to-camera R_i, t_i; the rotation is parameterised by two
 *              3-vectors (a1, a2) mapped to R = [b1 b2 b3] by Gram-Schmidt
 *              (the 6D representation the paper uses for global rotations);
 *   E_n        [t_hat]_x R_ij, R_ij = R_j R_i^T, t_ij = t_j - R_ij t_i,
 *              t_hat = t_ij / |t_ij|;
 *   residual   r_nm = x2~^T E_n x1~ (the epipolar error of eq. epipolar-objective);
 *   Gram       W_n = sum_m omega_nm w_nm w_nm^T, w_nm = flatten(x2~ x1~^T)
 *              (row-major: w[3a+b] = x2~[a] x1~[b]), App. B.6;
 *   loss       L = inv_Z * sum_n e_n^T W_n e_n, e_n = flatten(E_n) row-major
 *              (eq. epipolar-objective-l2 without the stray factor 2, which the
 *              derivation in App. B.6 does not produce);
 *   IRLS       omega = 1/max(|r|, delta) if |r| <= tau, else 0 (filtered),
 *              Z = number of matches with omega > 0 (Sec. 3.3, IRLS paragraph).
 *
 * Compact Gram layout ("W36").  W_{(ab),(cd)} = sum omega x2[a] x2[c] x1[b] x1[d]
 * depends on the unordered index pairs {a,c} and {b,d} only.  With the monomial
 * vector p(x) = (u^2, u v, v^2, u, v, 1) and q(a,c) the position of x~[a] x~[c]
 * in p (q(0,0)=0, q(0,1)=1, q(1,1)=2, q(0,2)=3, q(1,2)=4, q(2,2)=5), the pair's
 * Gram is stored as the 6x6 matrix
 *     W36[n][6*q2 + q1] = sum_m omega_nm p(x2_nm)[q2] p(x1_nm)[q1],
 * so W_{(ab),(cd)} = W36[n][6*q(a,c) + q(b,d)].  Entry 35 is sum_m omega_nm.
 *
 * Conventions for every call:
 *   - all array arguments are DEVICE pointers on the context's device, except
 *     where a comment says "host";  the caller owns every buffer;
 *   - calls are asynchronous on the given stream (NULL = the null stream);
 *     outputs are fully overwritten, never accumulated into;
 *   - argument validation happens on the host before any launch and returns
 *     FM_EINVAL / FM_ESHAPE / FM_EDTYPE with a message in fm_last_error();
 *     nothing is launched when a call returns an error;
 *   - results are deterministic: identical inputs on the same device and
 *     build give bit-identical outputs (fixed reduction orders, no
 *     floating-point atomics);
 *   - one context per host thread; a scene may be used from one stream at a
 *     time (it owns workspace the kernels write).
 */
#ifndef FASTMAP_HIP_H
#define FASTMAP_HIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fm_ctx fm_ctx;       /* device handle + last error message        */
typedef struct fm_scene fm_scene;   /* pair/match structure + derived index data */
typedef void* fm_stream;            /* a hipStream_t                             */

typedef enum {
  FM_OK = 0,
  FM_EINVAL = -1,        /* null pointer, bad scalar argument                      */
  FM_ESHAPE = -2,        /* inconsistent sizes, offsets or camera indices          */
  FM_EDTYPE = -3,        /* unsupported dtype                                      */
  FM_EHIP = -4,          /* a HIP runtime call failed                              */
  FM_ENOMEM = -5,        /* device allocation failed                               */
  FM_EDEVICE_CHECK = -6, /* fm_check: a kernel of the opt-in check mode flagged data */
  FM_ECOOP = -7          /* cooperative launch not possible for this size         */
} fm_status;

typedef enum { FM_F64 = 0, FM_F32 = 1, FM_BF16 = 2 } fm_dtype;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`. */
fm_status fm_create(fm_ctx** out, int device);
void fm_destroy(fm_ctx* ctx);
/* Message of the last failed call on this context (context-owned, valid until
 * the next call). */
const char* fm_last_error(const fm_ctx* ctx);
/* Library build string (host, static storage). */
const char* fm_version(void);

/* ------------------------------------------------------------------ check mode */

/* Data checks on the device (the conventions above: host-side argument
 * validation is always on; these look at the data the kernels read).  Off by
 * default.  While on, the calls below also run small scans whose findings
 * raise bits in a context-owned device flag:
 *   FM_CHECK_COORDS      a non-finite match coordinate (fm_build_pair_grams,
 *                        fm_reweight, fm_reweight_build: one extra pass over
 *                        the matches);
 *   FM_CHECK_PARAMS      non-finite pose parameters, or parameters whose
 *                        Gram-Schmidt or E_n is not finite (the IRLS calls
 *                        and fm_epipolar_loss_grad at their input poses,
 *                        fm_epipolar_solve at its final poses);
 *   FM_CHECK_DEGENERATE  a pair whose relative translation t_ij is 0 or at
 *                        most 1e-7 of |t_i| + |t_j| (below the resolution of
 *                        float32 parameters, so its direction is rounding
 *                        noise), at the same poses; a pair with t_ij exactly
 *                        0 adds 0 to the loss and gradient and gets r = 0;
 *   FM_CHECK_LOSS        a non-finite loss or gradient (fm_epipolar_loss_grad's
 *                        outputs, fm_epipolar_solve's loss trace).
 * The scans are enqueued on the call's stream after its own kernels, so they
 * see what the call read and wrote.  The calls still return FM_OK: the flag
 * is read by fm_check. */
typedef enum {
  FM_CHECK_COORDS = 1,
  FM_CHECK_PARAMS = 2,
  FM_CHECK_DEGENERATE = 4,
  FM_CHECK_LOSS = 8
} fm_check_bits;

/* Turn check mode on (enable != 0) or off.  The first enable allocates the
 * flag (4 bytes of device memory, freed by fm_destroy) and synchronises the
 * device. */
fm_status fm_set_check(fm_ctx* ctx, int enable);

/* Synchronise `stream`, read and clear the flag.  Returns FM_OK if no bit is
 * set (also when check mode was never enabled), else FM_EDEVICE_CHECK with
 * the checks named in fm_last_error().  flags (host, may be NULL) receives
 * the FM_CHECK_* bits that were set. */
fm_status fm_check(fm_ctx* ctx, fm_stream stream, uint32_t* flags);

/* ------------------------------------------------------------------ scene */

/* The problem structure of Sec. 3.3: P image pairs over N cameras and M
 * matches sorted by pair (CSR).
 *   pair_offsets [P+1] int64: off[0] = 0, nondecreasing, off[P] = M; the
 *                matches of pair n are rows off[n] .. off[n+1]-1;
 *   pair_cams    [P,2] int32: (i_n, j_n), 0 <= i_n, j_n < N, i_n != j_n;
 *   uv           [M,4] of `dtype` (FM_F64, FM_F32 or FM_BF16), row-major
 *                (u1, v1, u2, v2): normalised coordinates of x1 (image i_n)
 *                and x2 (image j_n).
 * The scene borrows these three arrays (they must outlive it and must not be
 * modified while it exists) and allocates its own index data and workspace
 * (work-item table, camera incidence lists, partial sums).  Creation validates
 * the offsets and camera indices on the device and synchronises `stream`;
 * a violation returns FM_ESHAPE.  P may be 0; M may be 0. */
fm_status fm_scene_create(fm_ctx* ctx, int64_t num_pairs, int64_t num_matches, int32_t num_cams,
                          const int64_t* pair_offsets, const int32_t* pair_cams,
                          const void* uv, fm_dtype dtype, fm_stream stream, fm_scene** out);
void fm_scene_destroy(fm_scene* scene);
/* Number of wavefronts the Gram pass launches (one per chunk of up to 1024
 * matches of a pair with more than 256 matches, plus one per group of four
 * smaller pairs); host value. */
int64_t fm_scene_work_items(const fm_scene* scene);

/* ------------------------------------------------------------------ a1: Gram */

/* build_pair_grams (App. B.6): W36[n] for every pair, with per-match weights
 * `weights` [M] float32 (NULL = all ones).
 *   W36_f64 [P,36] double  (may be NULL if W36_f32 is given)
 *   W36_f32 [P,36] float   (may be NULL if W36_f64 is given; the float copy
 *                           of the double result)
 * Per-match products and their sums within a work item are float32; the
 * work-item partials are added in float64 in work-item order.  A pair
 * without matches gets zeros. */
fm_status fm_build_pair_grams(fm_ctx* ctx, fm_scene* scene, const float* weights,
                              double* W36_f64, float* W36_f32, fm_stream stream);

/* ------------------------------------------------------------------ a2: IRLS */

/* reweight (Sec. 3.3, IRLS and filtering): at poses `params` [N,9] float32
 * (a1[3], a2[3], t[3] per camera) compute r = x2~^T E_n x1~ per match and
 * omega = 1/max(|r|, delta) if |r| <= tau else 0.
 *   weights_out [M] float (required), resid_out [M] float (NULL = not written),
 *   num_kept    [1] int64 device scalar: number of matches with omega > 0.
 * delta > 0 and tau > 0 are required.  A pair whose |t_ij| is 0 gives r = 0. */
fm_status fm_reweight(fm_ctx* ctx, fm_scene* scene, const float* params, float delta, float tau,
                      float* weights_out, float* resid_out, int64_t* num_kept, fm_stream stream);

/* reweight + build_pair_grams fused in one pass over the matches (no stored
 * weights): the Gram of the IRLS weights computed at `params`. */
fm_status fm_reweight_build(fm_ctx* ctx, fm_scene* scene, const float* params, float delta,
                            float tau, double* W36_f64, float* W36_f32, int64_t* num_kept,
                            fm_stream stream);

/* ------------------------------------------------------------------ a3+a4: loss, gradient */

/* epipolar_loss_grad (eq. epipolar-objective-l2 and its adjoint):
 *   W36     [P,36] compact Grams, `wdtype` FM_F64 or FM_F32;
 *   params  [N,9] float32;
 *   inv_Z   1/Z (host value), used when Z_dev is NULL;
 *   Z_dev   optional device int64 scalar Z (then inv_Z = 1/max(Z,1));
 *   loss    [1] double device scalar (NULL = not written);
 *   grad    [N,9] float32 dL/dparams (NULL = not written).
 * The per-pair essential matrix and quadratic form are evaluated in float64,
 * the Gram-Schmidt map and its adjoint in float64, the per-pair adjoint in
 * float32; per-camera sums run over each camera's pairs in pair order. */
fm_status fm_epipolar_loss_grad(fm_ctx* ctx, fm_scene* scene, const void* W36, fm_dtype wdtype,
                                const float* params, double inv_Z, const int64_t* Z_dev,
                                double* loss, float* grad, fm_stream stream);

/* ------------------------------------------------------------------ a5: Adam */

/* adam_step (Kingma & Ba with bias correction) over n float32 values:
 *   m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
 *   p <- p - lr * (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps)
 * step is 1-based (host).  lr points to device float32: one value
 * (lr_stride = 0) or n values (lr_stride = 1). */
fm_status fm_adam_step(fm_ctx* ctx, int64_t n, float* params, const float* grad, float* m,
                       float* v, int64_t step, const float* lr, int lr_stride, float beta1,
                       float beta2, float eps, fm_stream stream);

/* ------------------------------------------------------------------ fused loop */

typedef struct {
  float lr_rot;          /* lr0 on (a1, a2)                                   */
  float lr_t;            /* lr0 on t                                          */
  float lr_final_frac;   /* lr(k) = lr0 * frac^(k / lr_total_steps)           */
  float beta1, beta2, eps;
  int64_t lr_step0;      /* global step index of this call's first iteration  */
  int64_t lr_total_steps;/* length of the whole schedule (> 0)                */
  int64_t adam_step0;    /* Adam steps already taken on m, v (0 after a reset) */
  int32_t blocks;        /* workgroups (512 threads each) of the persistent
                            kernel (0 = automatic; capped at the co-resident
                            limit; > 0 also forces the pair-by-pair loop;
                            < 0 forces the camera-by-camera loop at any size,
                            automatic grid; fm_epipolar_solve only)          */
} fm_adam_cfg;

/* K iterations of {loss + gradient (as fm_epipolar_loss_grad), Adam update of
 * params} in ONE persistent cooperative kernel, with no host round trip
 * between iterations.  Two loops, same results up to the order of the float64
 * sums: pair by pair (a per-pair phase writes the records, a per-camera phase
 * sums them and steps Adam, grid-wide barriers between the two), or, for
 * graphs below 131,072 pairs when cfg->blocks is 0, camera by camera (one
 * wavefront per camera evaluates each of its pairs, so every pair is
 * evaluated from both ends, and one grid barrier per iteration; cfg->blocks
 * < 0 selects this loop at any size).  params, m, v [N,9] float32 are
 * updated in place.  loss_trace [K] double receives L before each update
 * (NULL = not written).  `cfg` is a host pointer. */
fm_status fm_epipolar_solve(fm_ctx* ctx, fm_scene* scene, const void* W36, fm_dtype wdtype,
                            float* params, float* m, float* v, int32_t K, const fm_adam_cfg* cfg,
                            double inv_Z, const int64_t* Z_dev, double* loss_trace,
                            fm_stream stream);

/* Failed grid barriers of the persistent launches (fm_epipolar_solve,
 * fm_translation_solve, fm_rotation_solve, fm_rotation_init) on this scene
 * since the last call (host value in *failures), then cleared.  A barrier wait is
 * bounded (about a second); if it expires, the launch stops at once and its
 * results are invalid.  Synchronises the device.  Not expected to be nonzero:
 * the cooperative launch makes every workgroup resident. */
fm_status fm_solve_barrier_failures(fm_ctx* ctx, fm_scene* scene, int64_t* failures);

/* ------------------------------------------------------------------ focal refinement */

/* Focal lengths refined inside epipolar adjustment (Sec. 3.3, the remark
 * after the IRLS paragraph: the focal lengths are built into the essential
 * matrices, which then are fundamental matrices).  The stored coordinates
 * are normalised by a focal estimate per camera; phi [N] float32 is the log
 * of each camera's refined focal over that estimate, S_i = diag(e^-phi_i,
 * e^-phi_i, 1), and F_n = S_j E_n S_i acts on the stored coordinates.  Each
 * pair's term is normalised by |F_n|_F^2 (without it, growing the scales
 * shrinks F toward a trivial zero of the algebraic loss; with unit relative
 * translation |E_n|_F^2 = 2, so at phi = 0 the loss is half the epipolar
 * one):
 *     L = inv_Z * sum_n f_n^T W_n f_n / f_n^T f_n,  f_n = flatten(F_n).
 * W36, wdtype, params, inv_Z, Z_dev as for fm_epipolar_loss_grad;
 *   loss [1] double, grad [N,9] float32 (dL/dparams), gphi [N] float32
 *   (dL/dphi); each NULL = not written.  A pair with |t_ij| = 0 adds
 *   nothing.  Float64 pair arithmetic, float32 records, fixed-order sums. */
fm_status fm_epipolar_focal_loss_grad(fm_ctx* ctx, fm_scene* scene, const void* W36, fm_dtype wdtype,
                                      const float* params, const float* phi, double inv_Z,
                                      const int64_t* Z_dev, double* loss, float* grad, float* gphi,
                                      fm_stream stream);

/* K Adam steps on the poses and the log focal scales of the loss above in
 * ONE persistent cooperative kernel, by the camera loop of
 * fm_epipolar_solve (one wavefront per camera evaluates each of its pairs,
 * one grid barrier per iteration).  params, m, v [N,9] and phi, m_phi,
 * v_phi [N] float32 are updated in place.  `cfg` (host) as for
 * fm_epipolar_solve (cfg->blocks ignored); lr_phi is the scales' initial
 * rate, decayed like the others.  W36, wdtype, inv_Z, Z_dev as for
 * fm_epipolar_focal_loss_grad.  loss_trace [K] double receives L before each
 * update (NULL = not written). */
fm_status fm_epipolar_focal_solve(fm_ctx* ctx, fm_scene* scene, const void* W36, fm_dtype wdtype,
                                  float* params, float* phi, float* m, float* v, float* m_phi,
                                  float* v_phi, int32_t K, const fm_adam_cfg* cfg, float lr_phi,
                                  double inv_Z, const int64_t* Z_dev, double* loss_trace,
                                  fm_stream stream);

/* ------------------------------------------------------------------ translation averaging */

/* Global translation averaging, the stage before epipolar adjustment
 * (Sec. 3.3 "Global Translation", eq. global-translation-objective, and the
 * appendix on multiple initialisations), on the scene's pair graph (its
 * matches are not used):
 *   target   d_n = o^{i->j} = -R_j^T t^{i->j}: world-to-camera rotation R_j of
 *            the pair's second camera and the pair's unit relative
 *            translation t^{i->j} (camera j's frame);
 *   loss     L_t(o) = (1/P) sum_n | (o_j - o_i)/|o_j - o_i| - d_n |_1 over the
 *            camera centres o; the L1 subgradient takes sign(0) = 0, and a
 *            pair whose two centres coincide adds nothing (P still counts it).
 * Independent runs (different initialisations) are processed together:
 * `runs` (1..64) copies of the centres laid out [runs, N, 3] float32.  The
 * calls below keep a per-scene workspace sized for the largest `runs` seen;
 * a call with more runs than before synchronises the device and grows it. */

/* dirs [P,3] float32 = -R_j^T t_rel[n] for each pair n, with R_j the
 * Gram-Schmidt rotation of params[j] (a1, a2; t ignored), params [N,9]
 * float32, t_rel [P,3] float32.  Float64 arithmetic. */
fm_status fm_translation_directions(fm_ctx* ctx, fm_scene* scene, const float* params,
                                    const float* t_rel, float* dirs, fm_stream stream);

/* L_t and its gradient for each run at centres [runs,N,3]:
 *   loss [runs] double (NULL = not written): the float32-rounded pair terms
 *        summed in float64;
 *   grad [runs,N,3] float32 (NULL = not written): per pair
 *        dL/ds = (I - u u^T) sign(u - d_n) / (P |s|), s = o_j - o_i, u = s/|s|
 *        (float64, stored float32), added to camera j and subtracted from
 *        camera i, summed per camera over its pairs in a fixed order. */
fm_status fm_translation_loss_grad(fm_ctx* ctx, fm_scene* scene, const float* dirs, int32_t runs,
                                   const float* centres, double* loss, float* grad, fm_stream stream);

/* K iterations of {gradient as fm_translation_loss_grad, Adam update of the
 * centres} for every run, in ONE persistent cooperative kernel, by the same
 * two loops as fm_epipolar_solve (camera by camera when cfg->blocks is 0,
 * at any graph size, else pair by pair).  centres, m, v
 * [runs,N,3] float32 are updated in place.  `cfg` (host) as for
 * fm_epipolar_solve, with lr_t the centres' initial rate (lr_rot unused).
 * loss_trace [runs,K] double receives L_t of each run before each update
 * (NULL = not written; tracing adds a workgroup reduction per run and
 * iteration).  Within the pair loop the centres do not depend on a forced
 * cfg->blocks; the two loops agree up to the order of their float64 sums. */
fm_status fm_translation_solve(fm_ctx* ctx, fm_scene* scene, const float* dirs, int32_t runs,
                               float* centres, float* m, float* v, int32_t K, const fm_adam_cfg* cfg,
                               double* loss_trace, fm_stream stream);

/* Merge of the runs (appendix on multiple initialisations): every run is
 * moved to its centroid and scaled to unit mean distance from it (a run
 * whose centres all coincide is only moved); each camera takes its aligned
 * centre from the run in which the mean L1 term of the camera's pairs is
 * lowest (the lowest run index among equals; a camera in no pair scores 0
 * and takes run 0).
 *   merged   [N,3] float32 (required);
 *   choice   [N] int32 run taken per camera (NULL = not written);
 *   cam_loss [runs,N] double the per-camera mean terms (NULL = not written).
 * Float64 arithmetic. */
fm_status fm_translation_merge(fm_ctx* ctx, fm_scene* scene, const float* dirs, int32_t runs,
                               const float* centres, float* merged, int32_t* choice, double* cam_loss,
                               fm_stream stream);

/* Relative-translation grid search (appendix on global translation,
 * "Relative Translation"), before translation averaging: for every pair,
 * with R_ij = R_j R_i^T from the rotations of params [N,9] float32 (a1, a2;
 * t ignored), the candidate t among cand [C,3] float64 (unit vectors,
 * device) with the lowest mean squared algebraic epipolar error
 *     t^T A_n t / |Q_n|,  A_n = B^T W_n B,  B[:, k] = flatten([e_k]_x R_ij)
 * (the squared residual x2~^T [t]_x R_ij x1~ averaged over the pair's
 * matches, from its Gram W36 [P,36] float64 as fm_build_pair_grams writes
 * it; |Q_n| from the scene's offsets).  The lowest candidate index wins among
 * equal errors.  The error is even in t, so the winner is negated when its
 * dot product with t_prior[n] ([P,3] float32) is negative; a pair without
 * matches keeps t_prior.  Float64 arithmetic.
 *   t_out   [P,3] float32 (required);
 *   best    [P] int32 winning candidate (-1: kept prior), NULL = not written;
 *   err_min [P] double its error, NULL = not written. */
fm_status fm_translation_search(fm_ctx* ctx, fm_scene* scene, const double* W36, const float* params,
                                const double* cand, int32_t C, const float* t_prior, float* t_out,
                                int32_t* best, double* err_min, fm_stream stream);

/* Epipolar parameters from the averaging stages' results: params9 [N,9]
 * float32 = (a1, a2, t = -R o) per camera, with (a1, a2) = params6 [N,6]
 * (rotation averaging's parameters) and o = centres [N,3] (translation
 * averaging's camera centres); R by Gram-Schmidt in float64. */
fm_status fm_poses_from_centres(fm_ctx* ctx, int32_t N, const float* params6, const float* centres,
                                float* params9, fm_stream stream);

/* ------------------------------------------------------------------ rotation averaging */

/* Global rotation averaging, the first pose stage (Sec. 3.3 "Global
 * Rotation", eq. rotation-objective and its geodesic distance; the appendix
 * on rotation initialisation), on the scene's pair graph (its matches are
 * not used):
 *   input    Rrel [P,9] float32, row-major: the measured relative rotation
 *            R^{i->j} of each pair (R_j ~ R^{i->j} R_i, world-to-camera);
 *   params   [N,6] float32 per camera (a1, a2): R_i = [b1 b2 b3] by
 *            Gram-Schmidt (the 6D representation);
 *   loss     L_R = (1/P) sum_n arccos((tr(R_j^T R^{i->j} R_i) - 1)/2), the
 *            argument clipped to [-1, 1]; where it is +-1 the pair adds no
 *            gradient.
 * The calls use the scene's pair-record and rotation workspace (the same
 * the epipolar calls use), so they must not overlap epipolar calls on the
 * scene. */

/* L_R at params (loss [1] double, NULL = not written) and dL_R/dparams
 * (grad [N,6] float32, NULL = not written): per pair in float64, records in
 * float32, summed per camera over its pairs in a fixed order, Gram-Schmidt
 * adjoint in float64. */
fm_status fm_rotation_loss_grad(fm_ctx* ctx, fm_scene* scene, const float* Rrel, const float* params,
                                double* loss, float* grad, fm_stream stream);

/* K iterations of {gradient as fm_rotation_loss_grad, Adam update of params}
 * in ONE persistent cooperative kernel, by the same two loops as
 * fm_epipolar_solve (camera by camera when cfg->blocks is 0, at any graph
 * size; the rotations of the current parameters are kept from one iteration
 * to the next).  params, m, v
 * [N,6] float32 are updated in place.  `cfg` (host) as for fm_epipolar_solve
 * with lr_rot the initial rate (lr_t unused).  loss_trace [K] double receives
 * L_R before each update (NULL = not written). */
fm_status fm_rotation_solve(fm_ctx* ctx, fm_scene* scene, const float* Rrel, float* params, float* m,
                            float* v, int32_t K, const fm_adam_cfg* cfg, double* loss_trace,
                            fm_stream stream);

/* Initial rotations by the column-wise least-squares problems of the
 * appendix on rotation initialisation:
 *   first columns  x = the unit vector minimising sum_n |x_j - R^{i->j} x_i|^2
 *                  over stacked 3-vectors (the eigenvector of the smallest
 *                  eigenvalue of its 3N x 3N matrix), then x_c / |x_c|;
 *   second columns the same with the pair term scaled 1/P plus
 *                  (1/N) sum_c (c1_c . y_c)^2, normalised per camera, made
 *                  orthogonal to c1_c by Gram-Schmidt;
 * params [N,6] float32 receives (c1, c2) per camera (the third column is
 * c1 x c2 by the 6D map).  Each eigenvector comes from at most `steps`
 * Lanczos steps (at most 3N and 4096) with full reorthogonalisation in one
 * persistent cooperative launch of `blocks` workgroups of 512 threads
 * (0 = automatic), started from start[col] ([2, 3N] float64, device; the
 * caller's random vectors), and the smallest eigenpair of the Lanczos
 * tridiagonal matrix; the steps end early once the Ritz pair's residual
 * bound |beta_k s_k| is below 1e-11 of |T| (checked every 10 steps).  info [4] double (device, NULL = not written): smallest eigenvalue
 * and steps taken, first then second problem.  The pair graph must be
 * connected (a camera in no pair makes the first problem's minimiser
 * meaningless); an empty graph returns FM_ESHAPE.  Uses a per-scene
 * workspace of (steps + 5) x 3N doubles, grown on demand (the growing call
 * synchronises the device). */
fm_status fm_rotation_init(fm_ctx* ctx, fm_scene* scene, const float* Rrel, const double* start,
                           int32_t steps, int32_t blocks, float* params, double* info, fm_stream stream);

/* ------------------------------------------------------------------ a9: learned weights */

/* Learned robust weights (an addition to the paper's IRLS, Sec. 3.3): a
 * 3 -> 64 -> 64 -> 1 MLP (ReLU, ReLU, sigmoid) maps per-match features to a
 * weight proposal in [0, 1].
 *
 * fm_match_features: at poses `params` [N,9] float32, per match
 *   feats[m] = (log max(|r|, delta), log |Q_n|, parallax angle in radians
 *               between the bearing rays R_i^T x1~ and R_j^T x2~)   [M,3] float32
 * (r in float64 as in fm_reweight). */
fm_status fm_match_features(fm_ctx* ctx, fm_scene* scene, const float* params, float delta,
                            float* feats, fm_stream stream);

/* Network weights, row-major [out, in], float32 device arrays:
 *   W1 [64,3], b1 [64], W2 [64,64], b2 [64], W3 [1,64], b3 [1];
 *   feat_mean [3], feat_std [3]: inputs are standardised (f - mean) / std. */
typedef struct {
  const float *W1, *b1, *W2, *b2, *W3, *b3, *feat_mean, *feat_std;
} fm_mlp;

typedef struct {
  float *W1, *b1, *W2, *b2, *W3, *b3;
} fm_mlp_grad;

/* out[m] = out_scale * sigmoid(z3[m]) for M matches.  The 64x64 layer runs
 * on MFMA with float16 operands and float32 accumulation; the first and last
 * layers in float32.  If `act` is given ([M,128] float16, device), the
 * post-ReLU activations of both hidden layers are kept for fm_mlp_backward. */
fm_status fm_mlp_forward(fm_ctx* ctx, int64_t M, const float* feats, const fm_mlp* w,
                         float out_scale, float* out, void* act, fm_stream stream);

/* Gradients of sum_m dout[m] * sigmoid(z3[m]) with respect to every weight
 * (fully overwritten, float32), from the activations kept by the forward
 * (z3 is recomputed from them).  Reductions over matches are deterministic:
 * per-wavefront partial sums, then a sum over wavefronts in a fixed order.
 * Uses a context-owned workspace that grows on demand (the first call with a
 * larger M synchronises `stream` and allocates). */
fm_status fm_mlp_backward(fm_ctx* ctx, int64_t M, const float* feats, const fm_mlp* w,
                          const void* act, const float* dout, fm_mlp_grad* g, fm_stream stream);

/* Change of every pair's relative pose between two parameter sets
 * params_a, params_b [N,9] float32 (the relative-pose error terms of the
 * paper's evaluation, Sec. 4.1 metrics; used as the convergence test of the
 * learned-weight form): with R_ij = R_j R_i^T and t_ij = t_j - R_ij t_i at
 * each set (Gram-Schmidt and all arithmetic in float64),
 *   rot_out [P] float32  angle of R_ij^a (R_ij^b)^T in degrees (NULL = not written);
 *   t_out   [P] float32  angle between t_ij^a and +-t_ij^b in degrees, the
 *                        smaller of the two signs (the epipolar objective
 *                        cannot tell t from -t); NULL = not written;
 *   counts  [2] int64    (device, required) the number of pairs whose
 *                        rotation change exceeds rot_deg, and whose
 *                        translation-direction change exceeds t_deg.
 * A pair with t_ij = 0 at either set has no direction and counts as a
 * translation change of 90 degrees.  Thresholds must be >= 0. */
fm_status fm_pose_change(fm_ctx* ctx, fm_scene* scene, const float* params_a, const float* params_b,
                         float rot_deg, float t_deg, float* rot_out, float* t_out, int64_t* counts,
                         fm_stream stream);

/* fm_mlp_backward without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses
 * that forbid hipMalloc): the same gradients, with the per-wavefront
 * gradient slots in a static device array of the library (512 slots of 4,481
 * floats, 9.2 MB, held by each GPU the library runs on until the process
 * ends) instead of a context workspace that grows on demand.  The launch is
 * capped at 128 workgroups of four wavefronts, so any M is accepted; up to
 * 8,192 matches it is fm_mlp_backward's launch and the results are
 * bit-identical, above it the float32 slot sums run in another order.
 * Every call on a GPU shares that GPU's array and fully rewrites the slots
 * it reads: calls that overlap on one GPU (two streams, two host threads)
 * race.  The first call on a device looks the array's device address up
 * (hipGetSymbolAddress); no call allocates. */
fm_status fm_mlp_backward_noalloc(fm_ctx* ctx, int64_t M, const float* feats, const fm_mlp* w,
                                  const void* act, const float* dout, fm_mlp_grad* g, fm_stream stream);

/* ------------------------------------------------------------------ launch timing */

/* Optional device-time measurement of the library's own launches (for
 * roofline reporting): while enabled, every launch of the kernels below is
 * bracketed by HIP events recorded on the launch's stream.
 *   FM_K_GRAM 0 (Gram / reweight pass over the matches), FM_K_SOLVE 1 (fused
 *   persistent loop), FM_K_ESSENTIALS 2, FM_K_FINALIZE 3, FM_K_PAIR 4 and
 *   FM_K_CAMERA 5 (the two kernels of fm_epipolar_loss_grad), FM_K_TA_SOLVE 6
 *   (persistent translation loop), FM_K_TA_PAIR 7 and FM_K_TA_CAMERA 8 (the
 *   two kernels of fm_translation_loss_grad), FM_K_RA_SOLVE 9 (persistent
 *   rotation loop), FM_K_RA_PAIR 10 and FM_K_RA_CAMERA 11 (the two kernels of
 *   fm_rotation_loss_grad), FM_K_RA_INIT 12 (rotation initialisation),
 *   FM_K_TS_SEARCH 13 (relative-translation grid search), FM_K_FO_PAIR 14 and
 *   FM_K_FO_CAMERA 15 (the two kernels of fm_epipolar_focal_loss_grad),
 *   FM_K_FO_SOLVE 16 (persistent focal loop), FM_K_GRAM_CALL 17 (the whole of
 *   one fm_build_pair_grams, fm_reweight or fm_reweight_build call: events on
 *   the call's stream before its first and after its last launch, so the
 *   interval includes the gaps between its kernels).
 * fm_profile_enable synchronises the device and clears earlier records;
 * fm_profile_read waits for the recorded events and returns the summed
 * elapsed milliseconds and the launch count of one kernel (host outputs). */
fm_status fm_profile_enable(fm_ctx* ctx, int enable);
fm_status fm_profile_read(fm_ctx* ctx, int kernel, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* FASTMAP_HIP_H */
