// Relative-translation grid search (FastMap, arXiv 2505.04612, appendix on
// global translation, "Relative Translation"): for every pair, with the
// relative rotation R_ij = R_j R_i^T of the global rotations, the unit vector
// among the candidates with the lowest mean squared algebraic epipolar error
// t^T A_n t / |Q_n|, A_n = B^T W_n B, B[:, k] = flatten([e_k]_x R_ij); the
// winner keeps the sign of the pair's prior estimate.
//
// One lane per (pair, slice of the candidates): S lanes share a pair and
// visit candidates slice, slice + S, ...; the candidates are staged in LDS
// tiles and read as broadcasts; the S lanes then combine their minima
// (value, then index) with a butterfly, so the lowest candidate index wins
// among equal errors whatever S is.
#include "fm_internal.h"

#include <cmath>

namespace {

constexpr int kTsTile = 1024;   // candidates per LDS tile: six monomials each (48 KB of float64)
// threads per workgroup (each workgroup stages every candidate once).  256
// rather than 512: the launch's workgroups then spread two or three to a
// CU instead of one or two, so the most loaded CUs carry 1.25x the mean
// instead of 1.67x (measured: medium graph 31.0 -> 29.3 us, the large
// street graph 525 -> 459 us, same results)
constexpr int kTsBlock = 256;

// A = B^T W B from the compact Gram (W_{(ab),(cd)} = W36[6 q(a,c) + q(b,d)])
// and R = R_ij, as its six distinct entries (A00, A11, A22, A01, A02, A12).
__device__ inline void pair_form(const double* __restrict__ w36, const double R[3][3], double A6[6]) {
  // B_k as 3x3: rows of [e_k]_x R
  double B[3][3][3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    B[0][0][b] = 0.0;      B[0][1][b] = -R[2][b]; B[0][2][b] = R[1][b];
    B[1][0][b] = R[2][b];  B[1][1][b] = 0.0;      B[1][2][b] = -R[0][b];
    B[2][0][b] = -R[1][b]; B[2][1][b] = R[0][b];  B[2][2][b] = 0.0;
  }
  // WB_l[(ab)] = sum_(cd) W[(ab),(cd)] B_l[c][d]
  double A[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      double wb[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double w = w36[6 * mono_q(a, c) + mono_q(b, d)];
#pragma unroll
          for (int l = 0; l < 3; ++l) wb[l] += w * B[l][c][d];
        }
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = 0; l < 3; ++l) A[k][l] += B[k][a][b] * wb[l];
    }
  A6[0] = A[0][0];
  A6[1] = A[1][1];
  A6[2] = A[2][2];
  A6[3] = A[0][1] + A[1][0];
  A6[4] = A[0][2] + A[2][0];
  A6[5] = A[1][2] + A[2][1];
}

__global__ __launch_bounds__(kTsBlock) void k_ts_search(const double* __restrict__ W36, const float* __restrict__ params,
                                                      const int32_t* __restrict__ cams,
                                                      const int64_t* __restrict__ offsets,
                                                      const double* __restrict__ cand, int32_t C,
                                                      const float* __restrict__ t_prior, int64_t P, int S,
                                                      float* __restrict__ t_out, int32_t* __restrict__ best_out,
                                                      double* __restrict__ err_out) {
  __shared__ double tile[kTsTile * 6];
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = gtid / S;
  const int slice = (int)(gtid % S);
  const bool live = n < P;
  double A6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t cnt = 0;
  if (live) {
    cnt = offsets[n + 1] - offsets[n];
    double a1[3], a2[3], t[3], Ri[3][3], Rj[3][3], R[3][3];
    load_pose(params, cams[2 * n], a1, a2, t);
    gs_matrix(gs_forward(a1, a2), Ri);
    load_pose(params, cams[2 * n + 1], a1, a2, t);
    gs_matrix(gs_forward(a1, a2), Rj);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) R[a][b] = Rj[a][0] * Ri[b][0] + Rj[a][1] * Ri[b][1] + Rj[a][2] * Ri[b][2];
    pair_form(W36 + 36 * n, R, A6);
  }
  double best_v = INFINITY;
  int best_i = 0x7fffffff;
  for (int base = 0; base < C; base += kTsTile) {
    const int len = C - base < kTsTile ? C - base : kTsTile;
    __syncthreads();
    // each candidate's monomials (x^2, y^2, z^2, xy, xz, yz), once per tile
    for (int k = threadIdx.x; k < len; k += blockDim.x) {
      const double x = cand[3 * (int64_t)(base + k)], y = cand[3 * (int64_t)(base + k) + 1],
                   z = cand[3 * (int64_t)(base + k) + 2];
      double* m = tile + 6 * k;
      m[0] = x * x;
      m[1] = y * y;
      m[2] = z * z;
      m[3] = x * y;
      m[4] = x * z;
      m[5] = y * z;
    }
    __syncthreads();
    if (live) {
      // four of this lane's candidates per step: their forms are independent
      // chains, evaluated as one expression each (the same rounding as one
      // at a time) and compared in candidate order (the same ties)
      int c = slice;
      for (; c + 3 * S < len; c += 4 * S) {
        double q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double* m = tile + 6 * (c + u * S);
          q[u] = A6[0] * m[0] + A6[1] * m[1] + A6[2] * m[2] + A6[3] * m[3] + A6[4] * m[4] + A6[5] * m[5];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (q[u] < best_v) {
            best_v = q[u];
            best_i = base + c + u * S;
          }
      }
      for (; c < len; c += S) {
        const double* m = tile + 6 * c;
        const double q = A6[0] * m[0] + A6[1] * m[1] + A6[2] * m[2] + A6[3] * m[3] + A6[4] * m[4] + A6[5] * m[5];
        if (q < best_v) {
          best_v = q;
          best_i = base + c;
        }
      }
    }
  }
  // combine the S lanes of a pair: lower value, then lower index
  for (int sh = 1; sh < S; sh <<= 1) {
    const double ov = __shfl_xor(best_v, sh);
    const int oi = __shfl_xor(best_i, sh);
    if (ov < best_v || (ov == best_v && oi < best_i)) {
      best_v = ov;
      best_i = oi;
    }
  }
  if (!live || slice != 0) return;
  double tp[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) tp[k] = (double)t_prior[3 * n + k];
  if (cnt == 0 || best_i >= C) {
#pragma unroll
    for (int k = 0; k < 3; ++k) t_out[3 * n + k] = (float)tp[k];
    if (best_out) best_out[n] = -1;
    if (err_out) err_out[n] = 0.0;
    return;
  }
  double tb[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) tb[k] = cand[3 * (int64_t)best_i + k];
  const double sgn = (tb[0] * tp[0] + tb[1] * tp[1] + tb[2] * tp[2]) < 0.0 ? -1.0 : 1.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) t_out[3 * n + k] = (float)(sgn * tb[k]);
  if (best_out) best_out[n] = best_i;
  if (err_out) err_out[n] = best_v / (double)cnt;
}

}  // namespace

extern "C" fm_status fm_translation_search(fm_ctx* ctx, fm_scene* s, const double* W36, const float* params,
                                           const double* cand, int32_t C, const float* t_prior, float* t_out,
                                           int32_t* best, double* err_min, fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  if (!s) return fm_fail(ctx, FM_EINVAL, "fm_translation_search: scene is NULL");
  if (s->ctx != ctx) return fm_fail(ctx, FM_EINVAL, "fm_translation_search: scene belongs to another context");
  if (C < 1) return fm_fail(ctx, FM_EINVAL, "fm_translation_search: no candidates");
  if (s->P == 0) return FM_OK;
  if (!W36 || !params || !cand || !t_prior || !t_out)
    return fm_fail(ctx, FM_EINVAL, "fm_translation_search: NULL argument");
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  // lanes per pair: enough (pair, slice) lanes for about two wavefronts per
  // SIMD (256 CUs x 4 SIMDs x 2 x 64 lanes), at most 64 (measured on the
  // medium graph, 4,096 candidates: 36.5 us; four wavefronts per SIMD with
  // 256-thread workgroups 39.7 us, one with 1,024-thread workgroups 56.6 us)
  int S = 1;
  while (S < 64 && s->P * S < (int64_t)256 * 4 * 2 * 64 && S < C) S <<= 1;
  const int64_t lanes = s->P * S;
  fm_timed timer(ctx, FM_K_TS_SEARCH, (hipStream_t)stream);
  hipLaunchKernelGGL(k_ts_search, dim3(grid_for(lanes, kTsBlock)), dim3(kTsBlock), 0, (hipStream_t)stream, W36, params,
                     s->pair_cams, s->offsets, cand, C, t_prior, s->P, S, t_out, best, err_min);
  FM_CHECK_LAUNCH(ctx);
  return FM_OK;
}
