// Loss, hand-written adjoint and Adam for epipolar adjustment: eq.
// (epipolar-objective-l2) evaluated per image pair from the compact Grams,
// its gradient with respect to the 6D rotation parameters and translations,
// and the fused persistent loop (Sec. 3.4's kernel fusion, re-designed as one
// cooperative kernel that also applies the Adam update).
//
// One iteration has two phases:
//   pair phase    one thread per image pair: E_n and W_n e_n in float64, the
//                 pair's loss, and the adjoint back to dL/dR and dL/dt of its
//                 two cameras (a 24-float record per pair);
//   camera phase  one 16-lane row of a wavefront per camera (four cameras
//                 per wavefront): the records of the camera's pairs are summed
//                 in a fixed order (lanes stride the camera's incidence list,
//                 then a fixed DPP tree inside the row), the Gram-Schmidt
//                 adjoint gives dL/d(a1, a2), and lanes 0..8 of the row apply
//                 Adam to one parameter each.
// The float64 quadratic form matters: near a minimum e^T W e is many orders
// of magnitude below |W| |e|^2, so float32 would cancel most of its digits.
#include "fm_internal.h"

template <typename WT>
__device__ inline double load_w(const WT* p, int k) {
  return (double)p[k];
}

// Loss term of pair n and what its adjoint needs: E_n at the current poses
// (`rot`, optional, holds each camera's rotation from Gram-Schmidt of the
// current parameters, so pairs need not repeat it) and g = W_n e_n, in
// float64.
struct PairEval {
  double Ri[3][3], Rj[3][3], Rij[3][3], th[3], ti[3], g[3][3];
  double ns, loss;
};

template <typename WT>
__device__ inline PairEval pair_eval(const float* __restrict__ params, const double* __restrict__ rot, int ci, int cj,
                                     const WT* __restrict__ W36, int64_t n) {
  PairEval e;
  double a1[3], a2[3], tj[3], E[3][3];
  if (rot) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      e.ti[k] = (double)params[(int64_t)ci * 9 + 6 + k];
      tj[k] = (double)params[(int64_t)cj * 9 + 6 + k];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      e.Ri[k / 3][k % 3] = rot[(int64_t)ci * 9 + k];
      e.Rj[k / 3][k % 3] = rot[(int64_t)cj * 9 + k];
    }
  } else {
    load_pose(params, ci, a1, a2, e.ti);
    gs_matrix(gs_forward(a1, a2), e.Ri);
    load_pose(params, cj, a1, a2, tj);
    gs_matrix(gs_forward(a1, a2), e.Rj);
  }
  e.ns = pair_essential(e.Ri, e.ti, e.Rj, tj, e.Rij, e.th, E);
  // g = W e with W_{(ab),(cd)} = W36[6 q(a,c) + q(b,d)]: walk the index
  // pairs (a, c) and read only the 6-entry row q(a,c) of the compact Gram
  // for each, so few Gram values are live at once
  const WT* Wn = W36 + n * 36;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) e.g[a][b] = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double row[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) row[k] = (double)Wn[6 * mono_q(a, c) + k];
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int d = 0; d < 3; ++d) e.g[a][b] = fma(row[mono_q(b, d)], E[c][d], e.g[a][b]);
    }
  e.loss = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) e.loss = fma(E[a][b], e.g[a][b], e.loss);
  return e;
}

// Loss term and adjoint record of pair n.  rec = [dL/dR_i (3x3 row-major),
// dL/dt_i, dL/dR_j, dL/dt_j] as float32.
template <typename WT>
__device__ inline double pair_loss_adjoint(const float* __restrict__ params, const double* __restrict__ rot, int ci,
                                           int cj, const WT* __restrict__ W36, int64_t n, double two_inv_Z,
                                           float* __restrict__ rec) {
  const PairEval e = pair_eval<WT>(params, rot, ci, cj, W36, n);
  if (!(e.ns > 0.0)) {
#pragma unroll
    for (int k = 0; k < 24; ++k) rec[k] = 0.0f;
    return 0.0;
  }
  // G = dL/dE = (2/Z) g ; A = G R_ij^T ; dR_ij = T^T G
  double G[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) G[a][b] = two_inv_Z * e.g[a][b];
  essential_adjoint(G, e.th, e.ns, e.Rij, e.Ri, e.Rj, e.ti, rec);
  return e.loss;
}

// Loss term of pair n and its adjoint in the fused loops' compact form
// (essential_adjoint_omega): om, dL/dt_i, dL/dt_j (all 0 for a degenerate
// pair).
template <typename WT>
__device__ inline double pair_loss_omega(const float* __restrict__ params, const double* __restrict__ rot, int ci,
                                         int cj, const WT* __restrict__ W36, int64_t n, double two_inv_Z,
                                         double om[3], double dti[3], double dtj[3]) {
  const PairEval e = pair_eval<WT>(params, rot, ci, cj, W36, n);
  if (!(e.ns > 0.0)) {
#pragma unroll
    for (int k = 0; k < 3; ++k) om[k] = dti[k] = dtj[k] = 0.0;
    return 0.0;
  }
  double G[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) G[a][b] = two_inv_Z * e.g[a][b];
  essential_adjoint_omega(G, e.th, e.ns, e.Rij, e.Ri, e.ti, om, dti, dtj);
  return e.loss;
}

// Pair phase over pairs [first, P) with stride `stride`; writes the records
// and returns this thread's loss sum (float64, in pair order).  The cameras
// of the first two pairs come in registers (ci0, cj0 and ci1, cj1), read
// once per solve.
template <typename WT>
__device__ inline double pair_phase(const float* params, const double* rot, const int32_t* cams, const WT* W36,
                                    int64_t P, double two_inv_Z, float* contrib, int64_t first, int64_t stride,
                                    int ci0, int cj0, int ci1 = 0, int cj1 = 0) {
  double sum = 0.0;
  for (int64_t n = first; n < P; n += stride) {
    float rec[24];
    const bool held0 = n == first, held1 = n == first + stride;
    const int ci = held0 ? ci0 : (held1 ? ci1 : cams[2 * n]), cj = held0 ? cj0 : (held1 ? cj1 : cams[2 * n + 1]);
    sum += pair_loss_adjoint<WT>(params, rot, ci, cj, W36, n, two_inv_Z, rec);
    float4* dst = reinterpret_cast<float4*>(contrib + n * 24);
#pragma unroll
    for (int k = 0; k < 6; ++k) dst[k] = make_float4(rec[4 * k], rec[4 * k + 1], rec[4 * k + 2], rec[4 * k + 3]);
  }
  return sum;
}

// Camera-major record layout of the pair loop: the 6 floats of item q of the
// incidence lists (a pair's side for one camera: its body-frame rotation
// gradient, -om for camera i and om for camera j, then dL/dt of that camera)
// at contrib + 6 q, so a camera's records are one contiguous run.  Pair phase
// as above, each side written to its slot (qi0, qj0 and qi1, qj1: slots of
// the first two pairs, held in registers).
template <typename WT>
__device__ inline double pair_phase_slots(const float* params, const double* rot, const int32_t* cams,
                                          const int32_t* pair_slot, const WT* W36, int64_t P, double two_inv_Z,
                                          float* contrib, int64_t first, int64_t stride, int ci0, int cj0, int ci1,
                                          int cj1, int qi0, int qj0, int qi1, int qj1) {
  double sum = 0.0;
  for (int64_t n = first; n < P; n += stride) {
    const bool held0 = n == first, held1 = n == first + stride;
    const int ci = held0 ? ci0 : (held1 ? ci1 : cams[2 * n]), cj = held0 ? cj0 : (held1 ? cj1 : cams[2 * n + 1]);
    const int qi = held0 ? qi0 : (held1 ? qi1 : pair_slot[2 * n]);
    const int qj = held0 ? qj0 : (held1 ? qj1 : pair_slot[2 * n + 1]);
    double om[3], dti[3], dtj[3];
    sum += pair_loss_omega<WT>(params, rot, ci, cj, W36, n, two_inv_Z, om, dti, dtj);
    float2* di = reinterpret_cast<float2*>(contrib + (int64_t)qi * 6);
    float2* dj = reinterpret_cast<float2*>(contrib + (int64_t)qj * 6);
    di[0] = make_float2((float)-om[0], (float)-om[1]);
    di[1] = make_float2((float)-om[2], (float)dti[0]);
    di[2] = make_float2((float)dti[1], (float)dti[2]);
    dj[0] = make_float2((float)om[0], (float)om[1]);
    dj[1] = make_float2((float)om[2], (float)dtj[0]);
    dj[2] = make_float2((float)dtj[1], (float)dtj[2]);
  }
  return sum;
}

// Incidence list of one camera as one wavefront reads it: the list bounds
// and the first two entries of this lane (q = lo + lane and lo + 64 + lane;
// -1 past the end).  Static during a solve, so the fused loop reads it once.
struct CamList {
  int lo, hi, it0, it1;
};

__device__ inline CamList cam_list(const int32_t* __restrict__ cam_ptr, const int32_t* __restrict__ cam_items, int c,
                                   int lane) {
  CamList L;
  L.lo = cam_ptr[c];
  L.hi = cam_ptr[c + 1];
  L.it0 = L.lo + lane < L.hi ? cam_items[L.lo + lane] : -1;
  L.it1 = L.lo + 64 + lane < L.hi ? cam_items[L.lo + 64 + lane] : -1;
  return L;
}

// Summed records of one camera over its incidence list, in every lane
// (lanes stride the list in pair order; wave_sum12 combines them).
__device__ inline void camera_sums(const CamList& L, const int32_t* __restrict__ cam_items,
                                   const float* __restrict__ contrib, int lane, double acc[12]) {
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  if (L.it0 >= 0) add_record(contrib, L.it0, acc);
  if (L.it1 >= 0) add_record(contrib, L.it1, acc);
  for (int q = L.lo + 128 + lane; q < L.hi; q += 64) add_record(contrib, cam_items[q], acc);
  wave_sum12(acc, lane);
}

// Gradient of camera c, computed by a whole wavefront; every lane returns
// dL/dtheta_c [9] (float64).
__device__ inline void camera_gradient(const float* __restrict__ params, const int32_t* __restrict__ cam_ptr,
                                       const int32_t* __restrict__ cam_items, const float* __restrict__ contrib,
                                       int c, int lane, double grad[9]) {
  double acc[12];
  camera_sums(cam_list(cam_ptr, cam_items, c, lane), cam_items, contrib, lane, acc);
  double a1[3], a2[3], t[3];
  load_pose(params, c, a1, a2, t);
  gs_adjoint(acc, a1, a2, grad);
}

// ------------------------------------------------------------------ standalone loss + gradient

template <typename WT>
__global__ __launch_bounds__(kBlock) void k_pair_phase(const float* __restrict__ params,
                                                       const int32_t* __restrict__ cams, const WT* __restrict__ W36,
                                                       int64_t P, double inv_Z, const int64_t* __restrict__ Z_dev,
                                                       float* __restrict__ contrib, double* __restrict__ loss_part) {
  __shared__ double lds[kBlock / 64];
  const double iz = Z_dev ? 1.0 / (double)(*Z_dev > 0 ? *Z_dev : 1) : inv_Z;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int ci0 = n < P ? cams[2 * n] : 0, cj0 = n < P ? cams[2 * n + 1] : 0;
  const double v =
      pair_phase(params, (const double*)nullptr, cams, W36, P, 2.0 * iz, contrib, n, P > 0 ? P : 1, ci0, cj0);
  const double t = block_sum(v, lds);
  if (threadIdx.x == 0) loss_part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_camera_grad(const float* __restrict__ params,
                                                        const int32_t* __restrict__ cam_ptr,
                                                        const int32_t* __restrict__ cam_items,
                                                        const float* __restrict__ contrib, int32_t N,
                                                        const double* __restrict__ loss_part, int64_t n_part,
                                                        double inv_Z, const int64_t* __restrict__ Z_dev,
                                                        float* __restrict__ grad, double* __restrict__ loss) {
  const int lane = threadIdx.x & 63;
  const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (loss && blockIdx.x == 0 && threadIdx.x == 0) {
    const double iz = Z_dev ? 1.0 / (double)(*Z_dev > 0 ? *Z_dev : 1) : inv_Z;
    double s = 0.0;
    for (int64_t k = 0; k < n_part; ++k) s += loss_part[k];
    *loss = s * iz;
  }
  if (c >= N || !grad) return;
  double g[9];
  camera_gradient(params, cam_ptr, cam_items, contrib, (int)c, lane, g);
  if (lane < 9) grad[c * 9 + lane] = (float)pick9(g, lane);
}

static fm_status check_w(fm_ctx* ctx, const char* fn, const void* W36, fm_dtype wdt, int64_t P) {
  if (!W36 && P > 0) return fm_fail(ctx, FM_EINVAL, "%s: W36 is NULL", fn);
  if (wdt != FM_F64 && wdt != FM_F32) return fm_fail(ctx, FM_EDTYPE, "%s: W36 must be FM_F64 or FM_F32", fn);
  return FM_OK;
}

extern "C" fm_status fm_epipolar_loss_grad(fm_ctx* ctx, fm_scene* s, const void* W36, fm_dtype wdt,
                                           const float* params, double inv_Z, const int64_t* Z_dev, double* loss,
                                           float* grad, fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  if (!s) return fm_fail(ctx, FM_EINVAL, "fm_epipolar_loss_grad: scene is NULL");
  if (s->ctx != ctx) return fm_fail(ctx, FM_EINVAL, "fm_epipolar_loss_grad: scene belongs to another context");
  fm_status rc = check_w(ctx, "fm_epipolar_loss_grad", W36, wdt, s->P);
  if (rc != FM_OK) return rc;
  if (!params && s->N > 0) return fm_fail(ctx, FM_EINVAL, "fm_epipolar_loss_grad: params is NULL");
  if (!Z_dev && !(inv_Z >= 0.0)) return fm_fail(ctx, FM_EINVAL, "fm_epipolar_loss_grad: inv_Z must be >= 0");
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const unsigned gp = grid_for(s->P > 0 ? s->P : 1, kBlock);
  {
  fm_timed timer(ctx, FM_K_PAIR, st);
  if (wdt == FM_F64)
    hipLaunchKernelGGL(k_pair_phase<double>, dim3(gp), dim3(kBlock), 0, st, params, s->pair_cams,
                       (const double*)W36, s->P, inv_Z, Z_dev, s->contrib, s->loss_part);
  else
    hipLaunchKernelGGL(k_pair_phase<float>, dim3(gp), dim3(kBlock), 0, st, params, s->pair_cams,
                       (const float*)W36, s->P, inv_Z, Z_dev, s->contrib, s->loss_part);
  }
  FM_CHECK_LAUNCH(ctx);
  const unsigned gc = grid_for((int64_t)(s->N > 0 ? s->N : 1) * 64, kBlock);
  {
  fm_timed timer(ctx, FM_K_CAMERA, st);
  hipLaunchKernelGGL(k_camera_grad, dim3(gc), dim3(kBlock), 0, st, params, s->cam_ptr, s->cam_items, s->contrib,
                     s->N, s->loss_part, (int64_t)gp, inv_Z, Z_dev, grad, loss);
  }
  FM_CHECK_LAUNCH(ctx);
  if (ctx->check) {
    // degenerate pairs and non-finite parameters at the input poses, then
    // the outputs themselves
    if ((rc = fm_launch_essentials(s, params, st)) != FM_OK) return rc;
    if ((rc = fm_check_finite(ctx, st, loss, 1, true, FM_CHECK_LOSS)) != FM_OK) return rc;
    if ((rc = fm_check_finite(ctx, st, grad, (int64_t)s->N * 9, false, FM_CHECK_LOSS)) != FM_OK) return rc;
  }
  return FM_OK;
}

// ------------------------------------------------------------------ Adam

__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, const float* __restrict__ lr, int lr_stride, double b1, double b2,
                       double eps, double bc1, double bc2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  float mk = m[k], vk = v[k];
  p[k] = adam_update(p[k], g[k], mk, vk, (double)lr[lr_stride ? k : 0], b1, b2, eps, bc1, bc2);
  m[k] = mk;
  v[k] = vk;
}

extern "C" fm_status fm_adam_step(fm_ctx* ctx, int64_t n, float* p, const float* g, float* m, float* v,
                                  int64_t step, const float* lr, int lr_stride, float beta1, float beta2, float eps,
                                  fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  if (n < 0) return fm_fail(ctx, FM_ESHAPE, "fm_adam_step: n < 0");
  if (n > 0 && (!p || !g || !m || !v || !lr)) return fm_fail(ctx, FM_EINVAL, "fm_adam_step: NULL argument");
  if (step < 1) return fm_fail(ctx, FM_EINVAL, "fm_adam_step: step is 1-based");
  if (lr_stride != 0 && lr_stride != 1) return fm_fail(ctx, FM_EINVAL, "fm_adam_step: lr_stride must be 0 or 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps >= 0.0f))
    return fm_fail(ctx, FM_EINVAL, "fm_adam_step: bad beta/eps");
  if (n == 0) return FM_OK;
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  const double bc1 = 1.0 - pow((double)beta1, (double)step), bc2 = 1.0 - pow((double)beta2, (double)step);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, (hipStream_t)stream, n, p, g, m, v, lr,
                     lr_stride, (double)beta1, (double)beta2, (double)eps, bc1, bc2);
  FM_CHECK_LAUNCH(ctx);
  return FM_OK;
}

// ------------------------------------------------------------------ fused persistent solve

// Re-arms the barriers before a launch: counts, generations and XCD
// registrations start at 0, and the launch's failure flag is cleared (a
// launch that ended on a failed barrier leaves it set).
__global__ void k_bar_reset(unsigned* __restrict__ bar) {
  if (threadIdx.x == 0) {
    bar[0] = 0u;
    bar[32] = 0u;
    bar[64] = 0u;
    bar[kBarTop] = 0u;
  }
  // grid_sync's per-XCD arrival counts, generations and workgroup
  // registrations
  if (threadIdx.x < kMaxXcd) {
    bar[kBarXcdCount + 32 * threadIdx.x] = 0u;
    bar[kBarXcdGen + 32 * threadIdx.x] = 0u;
    bar[kBarXcdReg + 32 * threadIdx.x] = 0u;
  }
}

hipError_t fm_bar_reset(unsigned* bar, hipStream_t st) {
  hipLaunchKernelGGL(k_bar_reset, dim3(1), dim3(64), 0, st, bar);
  return hipGetLastError();
}

struct SolveArgs {
  float* params;
  float* m;
  float* v;
  const int32_t* cams;
  const void* W36;
  const int32_t* cam_ptr;
  const int32_t* cam_items;
  float* contrib;
  double* loss_part;
  double* rot;
  double* loss_trace;
  unsigned* bar;
  const int64_t* Z_dev;
  double inv_Z;
  int64_t P;
  int32_t N;
  int32_t K;
  double lr_rot, lr_t, log_frac;
  double b1, b2, eps;
  int64_t lr_step0, lr_total, adam_step0;
  const int32_t* pair_slot;
};

// Record slots per lane that the pair loop's camera rows load in one round:
// 6 x 16 covers cameras of up to 96 pairs (slots past them are read in
// further rounds).
constexpr int kRowItems = 6;

// Summed records of one camera in every lane of its row, from the
// camera-major layout (slots lo..hi-1, 6 floats each): lane l16 takes slots
// lo + l16 + 16 j; the first NE of them are all loaded before any is added
// (so their loads are in flight together), then added in slot order, then
// the rest.  acc = (om, dL/dt) of the camera.
template <int NE>
__device__ inline void row_camera_sums_slots(int lo, int hi, const float* __restrict__ contrib, int lane,
                                             double (&acc)[6]) {
  const float2* c = reinterpret_cast<const float2*>(contrib);
  const int l16 = lane & 15;
  float2 r[NE][3];
#pragma unroll
  for (int j = 0; j < NE; ++j) {
    r[j][0] = r[j][1] = r[j][2] = make_float2(0.0f, 0.0f);
    const int q = lo + l16 + 16 * j;
    if (q < hi) {
      r[j][0] = c[(int64_t)q * 3];
      r[j][1] = c[(int64_t)q * 3 + 1];
      r[j][2] = c[(int64_t)q * 3 + 2];
    }
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) acc[k] = 0.0;
#pragma unroll
  for (int j = 0; j < NE; ++j) {
    acc[0] += r[j][0].x; acc[1] += r[j][0].y; acc[2] += r[j][1].x;
    acc[3] += r[j][1].y; acc[4] += r[j][2].x; acc[5] += r[j][2].y;
  }
  for (int q = lo + 16 * NE + l16; q < hi; q += 16) {
    const float2 a0 = c[(int64_t)q * 3], a1 = c[(int64_t)q * 3 + 1], a2 = c[(int64_t)q * 3 + 2];
    acc[0] += a0.x; acc[1] += a0.y; acc[2] += a1.x;
    acc[3] += a1.y; acc[4] += a2.x; acc[5] += a2.y;
  }
  row_sum6(acc, lane);
}

// Grid barrier of the fused loops: per-XCD (grid_sync) or flat
// (grid_barrier).
template <bool XS>
__device__ inline void loop_sync(GridBar& gb, XcdSync& xs) {
  if constexpr (XS)
    grid_sync(gb.bar, xs);
  else
    grid_barrier(gb);
}

template <typename WT, bool XS>
__global__ __launch_bounds__(kSolveBlock) void k_solve(SolveArgs a) {
  __shared__ double lds[kSolveBlock / 64];
  const double iz = a.Z_dev ? 1.0 / (double)(*a.Z_dev > 0 ? *a.Z_dev : 1) : a.inv_Z;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63;
  const int64_t gwave = gtid >> 6, nwaves = gsize >> 6;
  const WT* W36 = reinterpret_cast<const WT*>(a.W36);
  // static data of this thread's first two pairs (cameras and record slots)
  // and this row's first camera (its slot range), read once instead of once
  // per iteration
  const int ci0 = gtid < a.P ? a.cams[2 * gtid] : 0, cj0 = gtid < a.P ? a.cams[2 * gtid + 1] : 0;
  const int qi0 = gtid < a.P ? a.pair_slot[2 * gtid] : 0, qj0 = gtid < a.P ? a.pair_slot[2 * gtid + 1] : 0;
  const int64_t g1 = gtid + gsize;
  const int ci1 = g1 < a.P ? a.cams[2 * g1] : 0, cj1 = g1 < a.P ? a.cams[2 * g1 + 1] : 0;
  const int qi1 = g1 < a.P ? a.pair_slot[2 * g1] : 0, qj1 = g1 < a.P ? a.pair_slot[2 * g1 + 1] : 0;
  // cameras 4 gwave + row, then strided by 4 nwaves
  const int row = lane >> 4, l16 = lane & 15, base = lane & ~15;
  const int64_t c_first = 4 * gwave + row, c_stride = 4 * nwaves;
  const int lo0 = c_first < a.N ? a.cam_ptr[c_first] : 0, hi0 = c_first < a.N ? a.cam_ptr[c_first + 1] : 0;
  GridBar gb = grid_bar(a.bar);
  XcdSync xs = {};
  if constexpr (XS) xs = xcd_register(gb);
  StepSched sch(a.log_frac, a.lr_step0, a.lr_total, a.adam_step0, a.b1, a.b2);
  for (int k = 0; k < a.K; ++k) {
    // iteration 0 runs Gram-Schmidt per pair; later iterations read the
    // rotations the camera phase stored with the updated parameters
    const double v = pair_phase_slots<WT>(a.params, k > 0 ? a.rot : nullptr, a.cams, a.pair_slot, W36, a.P,
                                                2.0 * iz, a.contrib, gtid, gsize, ci0, cj0, ci1, cj1, qi0, qj0, qi1,
                                                qj1);
    const double t = block_sum(v, lds);
    if (threadIdx.x == 0) a.loss_part[blockIdx.x] = t;
    loop_sync<XS>(gb, xs);
    if (a.loss_trace && gtid == 0) {
      double s = 0.0;
      for (int b = 0; b < (int)gridDim.x; ++b) s += a.loss_part[b];
      a.loss_trace[k] = s * iz;
    }
    const double frac = sch.frac;
    const double bc1 = 1.0 - sch.p1, bc2 = 1.0 - sch.p2;
    sch.next();
    // the loop bound is uniform over the wavefront (rows past N idle), so
    // the row exchanges below always run with every lane present
    for (int64_t c0 = 4 * gwave; c0 < a.N; c0 += c_stride) {
      const int64_t c = c0 + row;
      const bool live = c < a.N;
      // parameters and moments first (they do not depend on the records),
      // so their loads overlap the record loads
      float p0 = 0.0f, mq = 0.0f, vq = 0.0f;
      // (m, v: only this lane reads and writes them during the launch)
      if (live && l16 < 9) {
        p0 = a.params[c * 9 + l16];
        mq = a.m[c * 9 + l16];
        vq = a.v[c * 9 + l16];
      }
      double acc6[6], acc[12];
      const bool first = c0 == 4 * gwave;
      const int lo = first ? lo0 : (live ? a.cam_ptr[c] : 0), hi = first ? hi0 : (live ? a.cam_ptr[c + 1] : 0);
      // Gram-Schmidt of the camera's own parameters ahead of the record
      // gather (it overlaps the record loads); a row without a camera has
      // zero parameters: keep its Gram-Schmidt away from 0/0 (its results
      // are not stored)
      double a1[3], a2[3], g[9];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        a1[j] = (double)__shfl(p0, base + j);
        a2[j] = (double)__shfl(p0, base + 3 + j);
      }
      if (!live) a1[0] = a2[1] = 1.0;
      const Gs f = gs_forward(a1, a2);
      row_camera_sums_slots<kRowItems>(lo, hi, a.contrib, lane, acc6);
      omega_grad(f, acc6, acc6 + 3, acc);
      gs_adjoint(acc, f, a2, g);
      // lanes 0..8 of the row update one parameter each
      float pq = 0.0f;
      if (live && l16 < 9) {
        const double lr = (l16 < 6 ? a.lr_rot : a.lr_t) * frac;
        pq = adam_update(p0, (float)pick9(g, l16), mq, vq, lr, a.b1, a.b2, a.eps, bc1, bc2);
        a.params[c * 9 + l16] = pq;
        a.m[c * 9 + l16] = mq;
        a.v[c * 9 + l16] = vq;
      }
      // rotation of the updated parameters for the next pair phase
      double n1[3], n2[3], R[3][3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        n1[j] = (double)__shfl(pq, base + j);
        n2[j] = (double)__shfl(pq, base + 3 + j);
      }
      if (!live) n1[0] = n2[1] = 1.0;
      gs_matrix(gs_forward(n1, n2), R);
      if (live && l16 < 9) {
        double rv = R[0][0];
#pragma unroll
        for (int j = 1; j < 9; ++j) rv = (l16 == j) ? R[j / 3][j % 3] : rv;
        a.rot[c * 9 + l16] = rv;
      }
    }
    loop_sync<XS>(gb, xs);
  }
}

// Camera-centric variant of the fused loop: one wavefront per camera; each
// lane evaluates one of the camera's pairs (its loss and the adjoint for the
// camera's own side, so every pair is evaluated twice, once from each end),
// the wavefront sums them in a fixed order and lanes 0..8 take the Adam
// step.  With no pair records to exchange, an iteration needs one grid
// barrier instead of two; the parameters and rotations a wavefront reads of
// other cameras are double-buffered by iteration parity so that each camera
// updates its own without a second barrier.
struct CamSolveArgs {
  float* params;       // buffer 0 (the caller's)
  float* params_alt;   // buffer 1 [N, 9]
  float* m;
  float* v;
  const int32_t* cams;
  const void* W36;
  const int32_t* cam_ptr;
  const int32_t* cam_items;
  double* rot;         // [2, N, 9]
  double* loss_part;   // [2, gridDim.x]
  double* loss_trace;
  unsigned* bar;
  const int64_t* Z_dev;
  double inv_Z;
  int64_t P;
  int32_t N;
  int32_t K;
  double lr_rot, lr_t, log_frac;
  double b1, b2, eps;
  int64_t lr_step0, lr_total, adam_step0;
};

// Gram-Schmidt of the parameters p0 held by lanes 0..5 of the wavefront (a2
// receives the second column's parameters).
__device__ inline Gs cam_gs(float p0, double a2[3]) {
  double a1[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    a1[j] = (double)__shfl(p0, j);
    a2[j] = (double)__shfl(p0, 3 + j);
  }
  return gs_forward(a1, a2);
}

// Rotation of an already formed Gram-Schmidt, stored by lanes 0..8 at
// rot[c] (written through to memory if WTS).
template <bool WTS>
__device__ inline void cam_store_gs(double* __restrict__ rot, int64_t c, const Gs& f, int lane) {
  double R[3][3];
  gs_matrix(f, R);
  if (lane < 9) {
    double rv = R[0][0];
#pragma unroll
    for (int j = 1; j < 9; ++j) rv = (lane == j) ? R[j / 3][j % 3] : rv;
    if constexpr (WTS)
      store_wt(&rot[c * 9 + lane], rv);
    else
      rot[c * 9 + lane] = rv;
  }
}

// Rotation of the parameters p0 held by lanes 0..5 of the wavefront, stored
// by lanes 0..8 at rot[c] (written through to memory if WTS).
template <bool WTS>
__device__ inline void cam_store_rot(double* __restrict__ rot, int64_t c, float p0, int lane) {
  double a2[3];
  cam_store_gs<WTS>(rot, c, cam_gs(p0, a2), lane);
}

template <typename WT, bool XS>
__global__ __launch_bounds__(kCamBlock) void k_solve_cam(CamSolveArgs a) {
  __shared__ double lds[kCamBlock / 64];
  const double iz = a.Z_dev ? 1.0 / (double)(*a.Z_dev > 0 ? *a.Z_dev : 1) : a.inv_Z;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63;
  const int64_t gwave = gtid >> 6, nwaves = gsize >> 6;
  const int kq = lane < 9 ? lane : 8;
  const WT* W36 = reinterpret_cast<const WT*>(a.W36);
  const int64_t NR = (int64_t)a.N * 9;
  // static data of the first 64 incidence entries of this wavefront's first
  // camera (one per lane: the pair, the camera's side, both cameras), read
  // once, so that each iteration's loads of that pass (poses, rotations,
  // Gram) all depend on registers only and are in flight together
  int n0 = -1, side0 = 0, ci0 = 0, cj0 = 0;
  if (gwave < a.N) {
    const int lo = a.cam_ptr[gwave], hi = a.cam_ptr[gwave + 1];
    if (lo + lane < hi) {
      const int item = a.cam_items[lo + lane];
      n0 = item >> 1;
      side0 = item & 1;
      ci0 = a.cams[2 * n0];
      cj0 = a.cams[2 * n0 + 1];
    }
  }
  // rotations of the initial parameters (buffer 0)
  for (int64_t c = gwave; c < a.N; c += nwaves) {
    const float p0 = a.params[c * 9 + kq];
    cam_store_rot<false>(a.rot, c, p0, lane);
  }
  // the wavefront's first camera stays in registers for the launch: its
  // parameters, Adam moments and their Gram-Schmidt, carried from one
  // iteration's update to the next instead of reloaded (after the barrier's
  // invalidation) and recomputed; its moments are stored once at the end
  const bool own = gwave < a.N;
  float p_own = 0.0f, m_own = 0.0f, v_own = 0.0f;
  double a2_own[3] = {0.0, 1.0, 0.0};
  Gs f_own{};
  if (own) {
    p_own = a.params[gwave * 9 + kq];
    m_own = a.m[gwave * 9 + kq];
    v_own = a.v[gwave * 9 + kq];
    f_own = cam_gs(p_own, a2_own);
  }
  GridBar gb = grid_bar(a.bar);
  XcdSync xs = {};
  if constexpr (XS)
    xs = xcd_register(gb);
  else
    grid_barrier(gb);
  StepSched sch(a.log_frac, a.lr_step0, a.lr_total, a.adam_step0, a.b1, a.b2);
  for (int k = 0; k < a.K; ++k) {
    const int rb = k & 1;
    const float* pr = rb ? a.params_alt : a.params;
    float* pw = rb ? a.params : a.params_alt;
    const double* rr = a.rot + rb * NR;
    double* rw = a.rot + (rb ^ 1) * NR;
    const double frac = sch.frac;
    const double bc1 = 1.0 - sch.p1, bc2 = 1.0 - sch.p2;
    sch.next();
    double lsum = 0.0;
    // the loop bound is uniform over the wavefront, so the wavefront sums
    // run with every lane present
    for (int64_t c = gwave; c < a.N; c += nwaves) {
      const int lo = a.cam_ptr[c], hi = a.cam_ptr[c + 1];
      // the camera's own parameters and moments (lanes 9..63 read entry 8;
      // m and v are read and written by this wavefront alone) and their
      // Gram-Schmidt, needed by the adjoint below: from registers for the
      // first camera, else loaded and formed ahead of the pair evaluations
      // (so that it overlaps their loads)
      const bool first_cam = c == gwave;
      float p0, mq, vq;
      double a2[3], g[9];
      Gs f;
      if (first_cam) {
        p0 = p_own;
        mq = m_own;
        vq = v_own;
#pragma unroll
        for (int j = 0; j < 3; ++j) a2[j] = a2_own[j];
        f = f_own;
      } else {
        p0 = pr[c * 9 + kq];
        mq = a.m[c * 9 + kq];
        vq = a.v[c * 9 + kq];
        f = cam_gs(p0, a2);
      }
      // this camera's side of each of its pairs: body-frame rotation
      // gradient (om for camera j, -om for camera i) and dL/dt
      double acc6[6], acc[12];
#pragma unroll
      for (int j = 0; j < 6; ++j) acc6[j] = 0.0;
      for (int q = lo + lane; q < hi; q += 64) {
        const bool first = c == gwave && q == lo + lane;
        const int item = first ? 0 : a.cam_items[q];
        const int64_t n = first ? n0 : item >> 1;
        const int side = first ? side0 : item & 1;
        const int ci = first ? ci0 : a.cams[2 * n], cj = first ? cj0 : a.cams[2 * n + 1];
        double om[3], dti[3], dtj[3];
        const double l = pair_loss_omega<WT>(pr, rr, ci, cj, W36, n, 2.0 * iz, om, dti, dtj);
        if (side == 0) lsum += l;   // each pair's loss once, from its first camera
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          acc6[j] += (double)(float)(side ? om[j] : -om[j]);
          acc6[3 + j] += (double)(float)(side ? dtj[j] : dti[j]);
        }
      }
      wave_sum6(acc6, lane);
      omega_grad(f, acc6, acc6 + 3, acc);
      gs_adjoint(acc, f, a2, g);
      const double lr = (lane < 6 ? a.lr_rot : a.lr_t) * frac;
      const float pq = adam_update(p0, (float)pick9(g, kq), mq, vq, lr, a.b1, a.b2, a.eps, bc1, bc2);
      // what other workgroups read (parameters, rotations, loss partials)
      // is written through to memory on the flat barrier's path; the Adam
      // moments stay with this wavefront
      if (lane < 9) {
        if constexpr (XS)
          pw[c * 9 + lane] = pq;
        else
          store_wt(&pw[c * 9 + lane], pq);
        if (!first_cam) {
          a.m[c * 9 + lane] = mq;
          a.v[c * 9 + lane] = vq;
        }
      }
      if (first_cam) {
        p_own = pq;
        m_own = mq;
        v_own = vq;
        f_own = cam_gs(pq, a2_own);
        cam_store_gs<!XS>(rw, c, f_own, lane);
      } else {
        cam_store_rot<!XS>(rw, c, pq, lane);
      }
    }
    if (a.loss_trace) {
      const double t = block_sum(lsum, lds);
      if (threadIdx.x == 0) {
        if constexpr (XS)
          a.loss_part[rb * gridDim.x + blockIdx.x] = t;
        else
          store_wt(&a.loss_part[rb * gridDim.x + blockIdx.x], t);
      }
    }
    if constexpr (XS)
      grid_sync(a.bar, xs);
    else
      grid_barrier_wt(gb);
    if (a.loss_trace && gtid == 0) {
      double sum = 0.0;
      for (int b = 0; b < (int)gridDim.x; ++b) sum += a.loss_part[rb * gridDim.x + b];
      a.loss_trace[k] = sum * iz;
    }
  }
  // the first camera's moments, kept in registers during the launch
  if (own && lane < 9) {
    a.m[gwave * 9 + lane] = m_own;
    a.v[gwave * 9 + lane] = v_own;
  }
  // after an odd number of iterations the latest parameters are in buffer 1
  if (a.K & 1) {
    for (int64_t c = gwave; c < a.N; c += nwaves)
      if (lane < 9) a.params[c * 9 + lane] = a.params_alt[c * 9 + lane];
  }
}

// Check mode after a fused solve: the final parameters and the loss trace
// finite, and no degenerate pair at the final poses.
static fm_status solve_checks(fm_ctx* ctx, fm_scene* s, const float* params, const double* loss_trace, int32_t K,
                              hipStream_t st) {
  if (!ctx->check) return FM_OK;
  fm_status rc = fm_check_finite(ctx, st, params, (int64_t)s->N * 9, false, FM_CHECK_PARAMS);
  if (rc == FM_OK) rc = fm_check_finite(ctx, st, loss_trace, K, true, FM_CHECK_LOSS);
  if (rc == FM_OK) rc = fm_launch_essentials(s, params, st);
  return rc;
}

// Co-resident workgroups of the fused loops: the smallest occupancy over
// every instantiation, times the CU count.
template <typename K>
static bool occ_min(K kernel, int block, int& per_cu) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block, 0) != hipSuccess) return false;
  if (n < per_cu) per_cu = n;
  return true;
}

int fm_solve_coop_blocks(fm_ctx* ctx, bool cam) {
  int per_cu = 1 << 20;
  const bool ok = cam ? occ_min(k_solve_cam<double, false>, kCamBlock, per_cu) &&
                            occ_min(k_solve_cam<float, false>, kCamBlock, per_cu) &&
                            occ_min(k_solve_cam<double, true>, kCamBlock, per_cu) &&
                            occ_min(k_solve_cam<float, true>, kCamBlock, per_cu)
                      : occ_min(k_solve<double, false>, kSolveBlock, per_cu) &&
                            occ_min(k_solve<float, false>, kSolveBlock, per_cu) &&
                            occ_min(k_solve<double, true>, kSolveBlock, per_cu) &&
                            occ_min(k_solve<float, true>, kSolveBlock, per_cu);
  return ok ? per_cu * ctx->num_cu : 0;
}

// Instantiation of a fused loop (camera or pair loop) for the Gram dtype
// and the barrier kind (per-XCD from kXcdSyncMinBlocks workgroups on).
static const void* loop_kernel(bool cam, fm_dtype wdt, int64_t blocks) {
  const bool xs = blocks >= kXcdSyncMinBlocks;
  if (cam) {
    if (wdt == FM_F64) return xs ? (const void*)k_solve_cam<double, true> : (const void*)k_solve_cam<double, false>;
    return xs ? (const void*)k_solve_cam<float, true> : (const void*)k_solve_cam<float, false>;
  }
  if (wdt == FM_F64) return xs ? (const void*)k_solve<double, true> : (const void*)k_solve<double, false>;
  return xs ? (const void*)k_solve<float, true> : (const void*)k_solve<float, false>;
}

extern "C" fm_status fm_epipolar_solve(fm_ctx* ctx, fm_scene* s, const void* W36, fm_dtype wdt, float* params,
                                       float* m, float* v, int32_t K, const fm_adam_cfg* cfg, double inv_Z,
                                       const int64_t* Z_dev, double* loss_trace, fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  if (!s) return fm_fail(ctx, FM_EINVAL, "fm_epipolar_solve: scene is NULL");
  if (s->ctx != ctx) return fm_fail(ctx, FM_EINVAL, "fm_epipolar_solve: scene belongs to another context");
  fm_status rc = check_w(ctx, "fm_epipolar_solve", W36, wdt, s->P);
  if (rc != FM_OK) return rc;
  if (!cfg || (s->N > 0 && (!params || !m || !v)))
    return fm_fail(ctx, FM_EINVAL, "fm_epipolar_solve: NULL argument");
  if (K < 0) return fm_fail(ctx, FM_EINVAL, "fm_epipolar_solve: K < 0");
  if (cfg->lr_total_steps <= 0 || cfg->lr_step0 < 0 || cfg->adam_step0 < 0 || !(cfg->lr_final_frac > 0.0f) ||
      !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f && cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f && cfg->eps >= 0.0f))
    return fm_fail(ctx, FM_EINVAL, "fm_epipolar_solve: bad Adam configuration");
  if (!Z_dev && !(inv_Z >= 0.0)) return fm_fail(ctx, FM_EINVAL, "fm_epipolar_solve: inv_Z must be >= 0");
  if (K == 0) return FM_OK;
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  // about one pair per thread or one 16-lane row per camera, capped at 16
  // workgroups below 32k pairs and at 192 above (each workgroup adds about
  // 0.02 us to each of the two grid barriers per iteration, measured, so
  // past these sizes a second round of pairs per thread is cheaper than more
  // workgroups), and at the co-resident limit
  int64_t want = grid_for(s->P, kSolveBlock);
  const int64_t want_c = grid_for((int64_t)s->N * 16, kSolveBlock);
  if (want_c > want) want = want_c;
  if (want > (s->P < 32768 ? 16 : 192)) want = s->P < 32768 ? 16 : 192;
  if (cfg->blocks > 0) want = cfg->blocks;
  if (want < 1) want = 1;
  if (want > s->coop_blocks) want = s->coop_blocks;
  if (want > s->loss_part_cap) return fm_fail(ctx, FM_ECOOP, "fm_epipolar_solve: loss workspace too small");
  SolveArgs a;
  a.params = params; a.m = m; a.v = v;
  a.cams = s->pair_cams; a.W36 = W36; a.cam_ptr = s->cam_ptr; a.cam_items = s->cam_items;
  a.contrib = s->contrib; a.loss_part = s->loss_part; a.rot = s->rot; a.loss_trace = loss_trace; a.Z_dev = Z_dev;
  a.bar = s->bar;
  a.inv_Z = inv_Z; a.P = s->P; a.N = s->N; a.K = K;
  a.lr_rot = cfg->lr_rot; a.lr_t = cfg->lr_t; a.log_frac = log((double)cfg->lr_final_frac);
  a.b1 = cfg->beta1; a.b2 = cfg->beta2; a.eps = cfg->eps;
  a.lr_step0 = cfg->lr_step0; a.lr_total = cfg->lr_total_steps; a.adam_step0 = cfg->adam_step0;
  a.pair_slot = s->pair_slot;
  void* args[] = {&a};
  hipLaunchKernelGGL(k_bar_reset, dim3(1), dim3(64), 0, (hipStream_t)stream, s->bar);
  FM_CHECK_LAUNCH(ctx);
  // automatic grid below kCamLoopMaxPairs, or cfg->blocks < 0: the
  // camera-centric loop, one barrier per iteration; a forced workgroup count
  // or a larger graph runs the pair loop
  int64_t want_cam = grid_for((int64_t)s->N * 64, kCamBlock);
  if (want_cam > s->coop_blocks_cam) want_cam = s->coop_blocks_cam;
  if ((cfg->blocks < 0 || (cfg->blocks == 0 && s->P < kCamLoopMaxPairs)) && 2 * want_cam <= s->loss_part_cap) {
    CamSolveArgs ca;
    ca.params = params; ca.params_alt = s->params_alt; ca.m = m; ca.v = v;
    ca.cams = s->pair_cams; ca.W36 = W36; ca.cam_ptr = s->cam_ptr; ca.cam_items = s->cam_items;
    ca.rot = s->rot; ca.loss_part = s->loss_part; ca.loss_trace = loss_trace; ca.bar = s->bar; ca.Z_dev = Z_dev;
    ca.inv_Z = inv_Z; ca.P = s->P; ca.N = s->N; ca.K = K;
    ca.lr_rot = a.lr_rot; ca.lr_t = a.lr_t; ca.log_frac = a.log_frac;
    ca.b1 = a.b1; ca.b2 = a.b2; ca.eps = a.eps;
    ca.lr_step0 = a.lr_step0; ca.lr_total = a.lr_total; ca.adam_step0 = a.adam_step0;
    void* cargs[] = {&ca};
    {
    fm_timed timer(ctx, FM_K_SOLVE, (hipStream_t)stream);
    hipError_t e = hipLaunchCooperativeKernel(loop_kernel(true, wdt, want_cam), dim3((unsigned)want_cam),
                                              dim3(kCamBlock), cargs, 0, (hipStream_t)stream);
    if (e != hipSuccess) return fm_fail(ctx, FM_ECOOP, "cooperative launch failed: %s", hipGetErrorString(e));
    }
    return solve_checks(ctx, s, params, loss_trace, K, (hipStream_t)stream);
  }
  {
  fm_timed timer(ctx, FM_K_SOLVE, (hipStream_t)stream);
  hipError_t e = hipLaunchCooperativeKernel(loop_kernel(false, wdt, want), dim3((unsigned)want), dim3(kSolveBlock),
                                            args, 0, (hipStream_t)stream);
  if (e != hipSuccess) return fm_fail(ctx, FM_ECOOP, "cooperative launch failed: %s", hipGetErrorString(e));
  }
  return solve_checks(ctx, s, params, loss_trace, K, (hipStream_t)stream);
}

extern "C" fm_status fm_solve_barrier_failures(fm_ctx* ctx, fm_scene* s, int64_t* failures) {
  if (!ctx) return FM_EINVAL;
  if (!s || !failures) return fm_fail(ctx, FM_EINVAL, "fm_solve_barrier_failures: NULL argument");
  if (s->ctx != ctx) return fm_fail(ctx, FM_EINVAL, "fm_solve_barrier_failures: scene belongs to another context");
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  FM_HIP_TRY(ctx, hipDeviceSynchronize());
  unsigned f = 0;
  FM_HIP_TRY(ctx, hipMemcpy(&f, s->bar + 96, sizeof(unsigned), hipMemcpyDeviceToHost));
  if (f) FM_HIP_TRY(ctx, hipMemset(s->bar + 96, 0, sizeof(unsigned)));
  *failures = (int64_t)f;
  return FM_OK;
}
