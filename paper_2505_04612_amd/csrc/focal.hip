// Focal-length refinement inside epipolar adjustment (FastMap, arXiv
// 2505.04612, Sec. 3.3: the focal lengths are built into the essential
// matrices, which then are fundamental matrices).  With coordinates
// normalised by a focal estimate per camera and a log focal scale phi_i
// (refined focal = estimate * exp(phi_i)), the pair's matrix acting on the
// stored coordinates is F_n = S_j E_n S_i, S = diag(e^-phi, e^-phi, 1), and
// the pair's term is normalised by |F_n|_F^2 (otherwise growing the scales
// shrinks F toward a trivial zero of the algebraic loss):
//     L = inv_Z * sum_n f_n^T W_n f_n / f_n^T f_n,  f_n = flatten(F_n).
// Pair phase: E_n and the quadratic form in float64, dL/dE back through the
// epipolar adjoint into the epipolar record layout, plus dL/dphi of both
// cameras; camera phase: the epipolar loop's row sums and Gram-Schmidt
// adjoint, and the sum of the focal records.
#include "fm_internal.h"

#include <cmath>

namespace {

// One pair's normalised term q = f^T W f / f^T f (returned) and, scaled by
// 2 iz, its adjoint: the epipolar record of both sides (rec [24]) and
// dL/dphi of both cameras.  A pair whose relative translation vanishes
// contributes nothing (q, rec and the focal terms are 0).
template <typename WT>
__device__ inline double fo_pair_terms(const double Ri[3][3], const double Rj[3][3], const double ti[3],
                                       const double tj[3], double phi_i, double phi_j,
                                       const WT* __restrict__ Wn, double iz, float* __restrict__ rec,
                                       double& dphi_i, double& dphi_j) {
  double Rij[3][3], th[3], E[3][3];
  const double ns = pair_essential(Ri, ti, Rj, tj, Rij, th, E);
  dphi_i = dphi_j = 0.0;
  if (!(ns > 0.0)) {
#pragma unroll
    for (int k = 0; k < 24; ++k) rec[k] = 0.0f;
    return 0.0;
  }
  const double ei = exp(-phi_i), ej = exp(-phi_j);
  const double si[3] = {ei, ei, 1.0}, sj[3] = {ej, ej, 1.0};
  double F[3][3], ff = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      F[a][b] = sj[a] * E[a][b] * si[b];
      ff += F[a][b] * F[a][b];
    }
  // g = W f with W_{(ab),(cd)} = W36[6 q(a,c) + q(b,d)]
  double g[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) g[a][b] = 0.0;
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
        for (int d = 0; d < 3; ++d) g[a][b] = fma(row[mono_q(b, d)], F[c][d], g[a][b]);
    }
  double num = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) num = fma(F[a][b], g[a][b], num);
  const double rff = 1.0 / ff;
  const double q = num * rff;
  // dL/dF = 2 iz (g - q F) / ff; dL/dE = dL/dF * S_j S_i; dF_ab/dphi_j =
  // -F_ab for a < 2, dF_ab/dphi_i = -F_ab for b < 2
  double G[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const double gf = 2.0 * iz * (g[a][b] - q * F[a][b]) * rff;
      G[a][b] = gf * sj[a] * si[b];
      if (a < 2) dphi_j -= gf * F[a][b];
      if (b < 2) dphi_i -= gf * F[a][b];
    }
  essential_adjoint(G, th, ns, Rij, Ri, Rj, ti, rec);
  return q;
}

template <typename WT>
__global__ __launch_bounds__(kBlock) void k_fo_pair(const float* __restrict__ params, const float* __restrict__ phi,
                                                    const int32_t* __restrict__ cams, const WT* __restrict__ W36,
                                                    int64_t P, double inv_Z, const int64_t* __restrict__ Z_dev,
                                                    float* __restrict__ contrib, float* __restrict__ fo_rec,
                                                    double* __restrict__ part) {
  __shared__ double lds[kBlock / 64];
  const double iz = Z_dev ? 1.0 / (double)(*Z_dev > 0 ? *Z_dev : 1) : inv_Z;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, gsize = (int64_t)gridDim.x * blockDim.x;
  double sum = 0.0;
  for (int64_t n = gtid; n < P; n += gsize) {
    const int ci = cams[2 * n], cj = cams[2 * n + 1];
    double a1[3], a2[3], ti[3], tj[3], Ri[3][3], Rj[3][3];
    load_pose(params, ci, a1, a2, ti);
    gs_matrix(gs_forward(a1, a2), Ri);
    load_pose(params, cj, a1, a2, tj);
    gs_matrix(gs_forward(a1, a2), Rj);
    float rec[24];
    double dpi, dpj;
    sum += fo_pair_terms(Ri, Rj, ti, tj, (double)phi[ci], (double)phi[cj], W36 + n * 36, iz, rec, dpi, dpj);
    float4* dst = reinterpret_cast<float4*>(contrib + n * 24);
#pragma unroll
    for (int k = 0; k < 6; ++k) dst[k] = make_float4(rec[4 * k], rec[4 * k + 1], rec[4 * k + 2], rec[4 * k + 3]);
    fo_rec[2 * n] = (float)dpi;
    fo_rec[2 * n + 1] = (float)dpj;
  }
  const double t = block_sum(sum, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = t * iz;
}

__global__ __launch_bounds__(kBlock) void k_fo_camera(const float* __restrict__ params,
                                                      const int32_t* __restrict__ cam_ptr,
                                                      const int32_t* __restrict__ cam_items,
                                                      const float* __restrict__ contrib,
                                                      const float* __restrict__ fo_rec, int32_t N,
                                                      float* __restrict__ grad, float* __restrict__ gphi) {
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = gtid >> 4;
  const int lane = threadIdx.x & 63, l16 = lane & 15;
  if (c >= N) return;   // whole rows leave together: the row exchanges stay within live rows
  const RowList L = row_list(cam_ptr, cam_items, (int)c, l16);
  double acc[12];
  row_camera_sums(L, cam_items, contrib, lane, acc);
  double a1[3], a2[3], t[3], g[9];
  load_pose(params, (int)c, a1, a2, t);
  gs_adjoint(acc, a1, a2, g);
  if (grad && l16 < 9) grad[9 * c + l16] = (float)pick9(g, l16);
  // focal records: the camera's own side of each of its pairs
  double f = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (L.it[j] >= 0) f += (double)fo_rec[L.it[j]];
  for (int q = L.lo + 64 + l16; q < L.hi; q += 16) f += (double)fo_rec[cam_items[q]];
#pragma unroll
  for (int sh = 8; sh >= 1; sh >>= 1) f += __shfl_xor(f, sh);
  if (gphi && l16 == 0) gphi[c] = (float)f;
}

__global__ void k_fo_loss_final(const double* __restrict__ part, int64_t nblocks, double* __restrict__ loss) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int64_t b = 0; b < nblocks; ++b) s += part[b];
  *loss = s;
}

// K Adam steps on poses and log focal scales in one persistent launch, by
// the camera loop of the epipolar solve: one wavefront per camera; each lane
// evaluates one of the camera's pairs and keeps its own side (the pose
// record, rounded to float32 as the records are, and dL/dphi); the
// wavefront sums them in a fixed order; lanes 0..8 step the pose and lane 9
// the scale.  Parameters, scales and rotations are double-buffered by
// iteration parity, so one grid barrier ends an iteration.
struct FoSolveArgs {
  float* params;       // buffer 0 [N, 9] (the caller's)
  float* params_alt;   // buffer 1 [N, 9]
  float* phi;          // buffer 0 [N] (the caller's)
  float* phi_alt;      // buffer 1 [N]
  float* m;            // [N, 9]
  float* v;
  float* m_phi;        // [N]
  float* v_phi;
  const int32_t* cams;
  const void* W36;
  const int32_t* cam_ptr;
  const int32_t* cam_items;
  double* rot;         // [2, N, 9]
  double* part;        // [2, gridDim.x]
  double* trace;
  unsigned* bar;
  const int64_t* Z_dev;
  double inv_Z;
  int32_t N;
  int32_t K;
  double lr_rot, lr_t, lr_phi, log_frac;
  double b1, b2, eps;
  int64_t lr_step0, lr_total, adam_step0;
};

// Rotation of the parameters p0 held by lanes 0..5, stored by lanes 0..8
// (written through to memory if WTS).
template <bool WTS>
__device__ inline void fo_store_rot(double* __restrict__ rot, int64_t c, float p0, int lane) {
  double a1[3], a2[3], R[3][3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    a1[j] = (double)__shfl(p0, j);
    a2[j] = (double)__shfl(p0, 3 + j);
  }
  gs_matrix(gs_forward(a1, a2), R);
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

template <typename WT>
__global__ __launch_bounds__(kSolveBlock) void k_fo_solve(FoSolveArgs a) {
  GridBar gb = grid_bar(a.bar);
  __shared__ double lds[kSolveBlock / 64];
  const double iz = a.Z_dev ? 1.0 / (double)(*a.Z_dev > 0 ? *a.Z_dev : 1) : a.inv_Z;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63;
  const int64_t gwave = gtid >> 6, nwaves = gsize >> 6;
  const int kq = lane < 9 ? lane : 8;
  const WT* W36 = reinterpret_cast<const WT*>(a.W36);
  const int64_t NR = (int64_t)a.N * 9;
  for (int64_t c = gwave; c < a.N; c += nwaves) fo_store_rot<false>(a.rot, c, a.params[c * 9 + kq], lane);
  grid_barrier(gb);
  // static data of the first 64 incidence entries of this wavefront's first
  // camera (one per lane: the entry and both cameras), read once
  int item0 = 0, ci0 = 0, cj0 = 0;
  if (gwave < a.N) {
    const int lo = a.cam_ptr[gwave], hi = a.cam_ptr[gwave + 1];
    if (lo + lane < hi) {
      item0 = a.cam_items[lo + lane];
      ci0 = a.cams[2 * (item0 >> 1)];
      cj0 = a.cams[2 * (item0 >> 1) + 1];
    }
  }
  StepSched sch(a.log_frac, a.lr_step0, a.lr_total, a.adam_step0, a.b1, a.b2);
  for (int k = 0; k < a.K; ++k) {
    const int rb = k & 1;
    const float* pr = rb ? a.params_alt : a.params;
    float* pw = rb ? a.params : a.params_alt;
    const float* fr = rb ? a.phi_alt : a.phi;
    float* fw = rb ? a.phi : a.phi_alt;
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
      const float p0 = pr[c * 9 + kq];
      float mq = a.m[c * 9 + kq], vq = a.v[c * 9 + kq];
      const float f0 = fr[c];
      float mf = a.m_phi[c], vf = a.v_phi[c];
      double acc[12], fsum = 0.0;
#pragma unroll
      for (int j = 0; j < 12; ++j) acc[j] = 0.0;
      for (int q = lo + lane; q < hi; q += 64) {
        // the lane's first entry of the wavefront's first camera from
        // registers (read once per launch), the others from memory
        const bool cached = c == gwave && q == lo + lane;
        const int item = cached ? item0 : a.cam_items[q];
        const int64_t n = item >> 1;
        const int side = item & 1;
        const int ci = cached ? ci0 : a.cams[2 * n], cj = cached ? cj0 : a.cams[2 * n + 1];
        double Ri[3][3], Rj[3][3], ti[3], tj[3];
#pragma unroll
        for (int e = 0; e < 9; ++e) {
          Ri[e / 3][e % 3] = rr[(int64_t)ci * 9 + e];
          Rj[e / 3][e % 3] = rr[(int64_t)cj * 9 + e];
        }
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          ti[e] = (double)pr[(int64_t)ci * 9 + 6 + e];
          tj[e] = (double)pr[(int64_t)cj * 9 + 6 + e];
        }
        float rec[24];
        double dpi, dpj;
        const double qn = fo_pair_terms(Ri, Rj, ti, tj, (double)fr[ci], (double)fr[cj], W36 + n * 36, iz, rec,
                                        dpi, dpj);
        if (side == 0) lsum += qn;   // each pair's term once, from its first camera
#pragma unroll
        for (int j = 0; j < 12; ++j) acc[j] += (double)(side ? rec[12 + j] : rec[j]);
        fsum += (double)(float)(side ? dpj : dpi);
      }
      wave_sum12(acc, lane);
#pragma unroll
      for (int sh = 32; sh >= 1; sh >>= 1) fsum += __shfl_xor(fsum, sh);
      double a1[3], a2[3], g[9];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        a1[j] = (double)__shfl(p0, j);
        a2[j] = (double)__shfl(p0, 3 + j);
      }
      gs_adjoint(acc, a1, a2, g);
      const double lr = (lane < 6 ? a.lr_rot : a.lr_t) * frac;
      const float pq = adam_update(p0, (float)pick9(g, kq), mq, vq, lr, a.b1, a.b2, a.eps, bc1, bc2);
      // parameters, scales, rotations and loss partials are read by other
      // workgroups after the barrier: written through to memory
      if (lane < 9) {
        store_wt(&pw[c * 9 + lane], pq);
        a.m[c * 9 + lane] = mq;
        a.v[c * 9 + lane] = vq;
      }
      if (lane == 9) {
        store_wt(&fw[c], adam_update(f0, (float)fsum, mf, vf, a.lr_phi * frac, a.b1, a.b2, a.eps, bc1, bc2));
        a.m_phi[c] = mf;
        a.v_phi[c] = vf;
      }
      fo_store_rot<true>(rw, c, pq, lane);
    }
    if (a.trace) {
      const double t = block_sum(lsum, lds);
      if (threadIdx.x == 0) store_wt(&a.part[rb * gridDim.x + blockIdx.x], t);
    }
    grid_barrier_wt(gb);
    if (a.trace && gtid == 0) {
      double t = 0.0;
      for (int b = 0; b < (int)gridDim.x; ++b) t += a.part[rb * gridDim.x + b];
      a.trace[k] = t * iz;
    }
  }
  // after an odd number of iterations the latest values are in buffer 1
  if (a.K & 1) {
    for (int64_t c = gwave; c < a.N; c += nwaves) {
      if (lane < 9) a.params[c * 9 + lane] = a.params_alt[c * 9 + lane];
      if (lane == 9) a.phi[c] = a.phi_alt[c];
    }
  }
}

}  // namespace

extern "C" fm_status fm_epipolar_focal_loss_grad(fm_ctx* ctx, fm_scene* s, const void* W36, fm_dtype wdt,
                                                 const float* params, const float* phi, double inv_Z,
                                                 const int64_t* Z_dev, double* loss, float* grad, float* gphi,
                                                 fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  if (!s) return fm_fail(ctx, FM_EINVAL, "fm_epipolar_focal_loss_grad: scene is NULL");
  if (s->ctx != ctx) return fm_fail(ctx, FM_EINVAL, "fm_epipolar_focal_loss_grad: scene belongs to another context");
  if (wdt != FM_F64 && wdt != FM_F32) return fm_fail(ctx, FM_EDTYPE, "fm_epipolar_focal_loss_grad: W36 must be F64 or F32");
  if ((s->P > 0 && !W36) || (s->N > 0 && (!params || !phi)))
    return fm_fail(ctx, FM_EINVAL, "fm_epipolar_focal_loss_grad: NULL argument");
  if (!Z_dev && !(inv_Z >= 0.0)) return fm_fail(ctx, FM_EINVAL, "fm_epipolar_focal_loss_grad: inv_Z must be >= 0");
  if (!loss && !grad && !gphi) return FM_OK;
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const unsigned gp = grid_for(s->P > 0 ? s->P : 1, kBlock);
  {
    fm_timed timer(ctx, FM_K_FO_PAIR, st);
    if (wdt == FM_F64)
      hipLaunchKernelGGL(k_fo_pair<double>, dim3(gp), dim3(kBlock), 0, st, params, phi, s->pair_cams,
                         (const double*)W36, s->P, inv_Z, Z_dev, s->contrib, s->fo_rec, s->loss_part);
    else
      hipLaunchKernelGGL(k_fo_pair<float>, dim3(gp), dim3(kBlock), 0, st, params, phi, s->pair_cams,
                         (const float*)W36, s->P, inv_Z, Z_dev, s->contrib, s->fo_rec, s->loss_part);
    FM_CHECK_LAUNCH(ctx);
  }
  if (loss) {
    hipLaunchKernelGGL(k_fo_loss_final, dim3(1), dim3(64), 0, st, s->loss_part, (int64_t)gp, loss);
    FM_CHECK_LAUNCH(ctx);
  }
  if ((grad || gphi) && s->N > 0) {
    fm_timed timer(ctx, FM_K_FO_CAMERA, st);
    hipLaunchKernelGGL(k_fo_camera, dim3(grid_for((int64_t)s->N * 16, kBlock)), dim3(kBlock), 0, st, params,
                       s->cam_ptr, s->cam_items, s->contrib, s->fo_rec, s->N, grad, gphi);
    FM_CHECK_LAUNCH(ctx);
  }
  return FM_OK;
}

extern "C" fm_status fm_epipolar_focal_solve(fm_ctx* ctx, fm_scene* s, const void* W36, fm_dtype wdt, float* params,
                                             float* phi, float* m, float* v, float* m_phi, float* v_phi, int32_t K,
                                             const fm_adam_cfg* cfg, float lr_phi, double inv_Z,
                                             const int64_t* Z_dev, double* loss_trace, fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  if (!s) return fm_fail(ctx, FM_EINVAL, "fm_epipolar_focal_solve: scene is NULL");
  if (s->ctx != ctx) return fm_fail(ctx, FM_EINVAL, "fm_epipolar_focal_solve: scene belongs to another context");
  if (wdt != FM_F64 && wdt != FM_F32) return fm_fail(ctx, FM_EDTYPE, "fm_epipolar_focal_solve: W36 must be F64 or F32");
  if (!cfg || (s->P > 0 && !W36) || (s->N > 0 && (!params || !phi || !m || !v || !m_phi || !v_phi)))
    return fm_fail(ctx, FM_EINVAL, "fm_epipolar_focal_solve: NULL argument");
  if (K < 0) return fm_fail(ctx, FM_EINVAL, "fm_epipolar_focal_solve: K < 0");
  if (!Z_dev && !(inv_Z >= 0.0)) return fm_fail(ctx, FM_EINVAL, "fm_epipolar_focal_solve: inv_Z must be >= 0");
  if (cfg->lr_total_steps <= 0 || cfg->lr_step0 < 0 || cfg->adam_step0 < 0 || !(cfg->lr_final_frac > 0.0f) ||
      !(cfg->lr_rot >= 0.0f) || !(cfg->lr_t >= 0.0f) || !(lr_phi >= 0.0f) ||
      !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f && cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f && cfg->eps >= 0.0f))
    return fm_fail(ctx, FM_EINVAL, "fm_epipolar_focal_solve: bad Adam configuration");
  if (K == 0 || s->N == 0) return FM_OK;
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  if (s->fo_coop_blocks <= 0) {
    int pc64 = 0, pc32 = 0;
    FM_HIP_TRY(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc64, k_fo_solve<double>, kSolveBlock, 0));
    FM_HIP_TRY(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc32, k_fo_solve<float>, kSolveBlock, 0));
    s->fo_coop_blocks = (pc64 < pc32 ? pc64 : pc32) * ctx->num_cu;
    if (s->fo_coop_blocks <= 0) return fm_fail(ctx, FM_ECOOP, "cannot size the cooperative focal kernel");
  }
  // one wavefront per camera up to the co-resident limit (cameras strided
  // beyond it); two sets of loss partials
  const CamGrid cg = cam_grid(s->N, s->fo_coop_blocks, ctx->num_cu);
  int64_t want = cg.blocks;
  if (2 * want > s->loss_part_cap) want = s->loss_part_cap / 2;
  if (want < 1) return fm_fail(ctx, FM_ECOOP, "fm_epipolar_focal_solve: no room for the loss partials");
  FoSolveArgs a;
  a.params = params; a.params_alt = s->params_alt; a.phi = phi; a.phi_alt = s->params_alt + 9 * (int64_t)s->N;
  a.m = m; a.v = v; a.m_phi = m_phi; a.v_phi = v_phi;
  a.cams = s->pair_cams; a.W36 = W36; a.cam_ptr = s->cam_ptr; a.cam_items = s->cam_items;
  a.rot = s->rot; a.part = s->loss_part; a.trace = loss_trace; a.bar = s->bar; a.Z_dev = Z_dev;
  a.inv_Z = inv_Z; a.N = s->N; a.K = K;
  a.lr_rot = cfg->lr_rot; a.lr_t = cfg->lr_t; a.lr_phi = lr_phi; a.log_frac = log((double)cfg->lr_final_frac);
  a.b1 = cfg->beta1; a.b2 = cfg->beta2; a.eps = cfg->eps;
  a.lr_step0 = cfg->lr_step0; a.lr_total = cfg->lr_total_steps; a.adam_step0 = cfg->adam_step0;
  void* args[] = {&a};
  FM_HIP_TRY(ctx, fm_bar_reset(s->bar, st));
  fm_timed timer(ctx, FM_K_FO_SOLVE, st);
  hipError_t e = wdt == FM_F64 ? hipLaunchCooperativeKernel((const void*)k_fo_solve<double>, dim3((unsigned)want),
                                                           dim3(cg.threads), args, 0, st)
                               : hipLaunchCooperativeKernel((const void*)k_fo_solve<float>, dim3((unsigned)want),
                                                           dim3(cg.threads), args, 0, st);
  if (e != hipSuccess) return fm_fail(ctx, FM_ECOOP, "cooperative launch failed: %s", hipGetErrorString(e));
  return FM_OK;
}
