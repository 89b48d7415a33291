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
    double a1[3], a2[3], ti[3], tj[3], Ri[3][3], Rj[3][3], Rij[3][3], th[3], E[3][3];
    load_pose(params, ci, a1, a2, ti);
    gs_matrix(gs_forward(a1, a2), Ri);
    load_pose(params, cj, a1, a2, tj);
    gs_matrix(gs_forward(a1, a2), Rj);
    const double ns = pair_essential(Ri, ti, Rj, tj, Rij, th, E);
    float rec[24];
    float4* dst = reinterpret_cast<float4*>(contrib + n * 24);
    if (!(ns > 0.0)) {
#pragma unroll
      for (int k = 0; k < 6; ++k) dst[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      fo_rec[2 * n] = 0.0f;
      fo_rec[2 * n + 1] = 0.0f;
      continue;
    }
    const double ei = exp(-(double)phi[ci]), ej = exp(-(double)phi[cj]);
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
    const WT* Wn = W36 + n * 36;
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
    sum += q;
    // dL/dF = 2 iz (g - q F) / ff; dL/dE = dL/dF * S_j S_i; dF_ab/dphi_j =
    // -F_ab for a < 2, dF_ab/dphi_i = -F_ab for b < 2
    double G[3][3], dphi_i = 0.0, dphi_j = 0.0;
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
#pragma unroll
    for (int k = 0; k < 6; ++k) dst[k] = make_float4(rec[4 * k], rec[4 * k + 1], rec[4 * k + 2], rec[4 * k + 3]);
    fo_rec[2 * n] = (float)dphi_i;
    fo_rec[2 * n + 1] = (float)dphi_j;
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
