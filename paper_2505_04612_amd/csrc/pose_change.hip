// Per-pair change of the relative poses between two parameter sets: the
// convergence test of the learned-weight form (how far a plain IRLS loop
// moves each pair's relative rotation and translation direction), in the
// relative-pose error terms of the paper's evaluation (Sec. 4.1 metrics).
#include "fm_internal.h"

// Angle (degrees) of Qa Qb^T for two rotations, from its skew part and trace
// (atan2, accurate at small angles).
__device__ inline double rot_angle_deg(const double Qa[3][3], const double Qb[3][3]) {
  double D[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) D[r][c] = Qa[r][0] * Qb[c][0] + Qa[r][1] * Qb[c][1] + Qa[r][2] * Qb[c][2];
  const double cs = 0.5 * (D[0][0] + D[1][1] + D[2][2] - 1.0);
  const double ax = D[2][1] - D[1][2], ay = D[0][2] - D[2][0], az = D[1][0] - D[0][1];
  return atan2(0.5 * sqrt(ax * ax + ay * ay + az * az), cs) * (180.0 / M_PI);
}

// One thread per pair: R_ij and t_ij at both parameter sets (float64
// Gram-Schmidt), the rotation change and the translation-direction change
// with the sign of t ignored (the epipolar objective cannot see it); pairs
// over either threshold are counted with a wavefront ballot.
__global__ __launch_bounds__(kBlock) void k_pose_change(const float* __restrict__ pa, const float* __restrict__ pb,
                                                        const int32_t* __restrict__ cams, int64_t P, double rot_deg,
                                                        double t_deg, float* __restrict__ rot_out,
                                                        float* __restrict__ t_out,
                                                        unsigned long long* __restrict__ counts) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool over_r = false, over_t = false;
  if (n < P) {
    const int ci = cams[2 * n], cj = cams[2 * n + 1];
    double Q[2][3][3], u[2][3], ns[2];
    for (int k = 0; k < 2; ++k) {
      const float* prm = k ? pb : pa;
      double a1[3], a2[3], ti[3], tj[3], Ri[3][3], Rj[3][3], th[3], E[3][3];
      load_pose(prm, ci, a1, a2, ti);
      gs_matrix(gs_forward(a1, a2), Ri);
      load_pose(prm, cj, a1, a2, tj);
      gs_matrix(gs_forward(a1, a2), Rj);
      ns[k] = pair_essential(Ri, ti, Rj, tj, Q[k], th, E);
      for (int a = 0; a < 3; ++a) u[k][a] = th[a];
    }
    const double dr = rot_angle_deg(Q[0], Q[1]);
    const double cx = u[0][1] * u[1][2] - u[0][2] * u[1][1], cy = u[0][2] * u[1][0] - u[0][0] * u[1][2],
                 cz = u[0][0] * u[1][1] - u[0][1] * u[1][0];
    // a pair without a direction at either set counts as 90 degrees
    const double dt =
        (ns[0] > 0.0 && ns[1] > 0.0)
            ? atan2(sqrt(cx * cx + cy * cy + cz * cz), fabs(u[0][0] * u[1][0] + u[0][1] * u[1][1] + u[0][2] * u[1][2])) *
                  (180.0 / M_PI)
            : 90.0;
    if (rot_out) rot_out[n] = (float)dr;
    if (t_out) t_out[n] = (float)dt;
    over_r = dr > rot_deg;
    over_t = dt > t_deg;
  }
  const unsigned long long br = __ballot(over_r), bt = __ballot(over_t);
  if ((threadIdx.x & 63) == 0) {
    if (br) atomicAdd(&counts[0], (unsigned long long)__popcll(br));
    if (bt) atomicAdd(&counts[1], (unsigned long long)__popcll(bt));
  }
}

__global__ void k_zero_counts(unsigned long long* __restrict__ counts) {
  if (threadIdx.x < 2) counts[threadIdx.x] = 0ull;
}

extern "C" fm_status fm_pose_change(fm_ctx* ctx, fm_scene* s, const float* params_a, const float* params_b,
                                    float rot_deg, float t_deg, float* rot_out, float* t_out, int64_t* counts,
                                    fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  if (!s) return fm_fail(ctx, FM_EINVAL, "fm_pose_change: scene is NULL");
  if (s->ctx != ctx) return fm_fail(ctx, FM_EINVAL, "fm_pose_change: scene belongs to another context");
  if (!counts) return fm_fail(ctx, FM_EINVAL, "fm_pose_change: counts is NULL");
  if (s->N > 0 && (!params_a || !params_b)) return fm_fail(ctx, FM_EINVAL, "fm_pose_change: params is NULL");
  if (!(rot_deg >= 0.0f) || !(t_deg >= 0.0f)) return fm_fail(ctx, FM_EINVAL, "fm_pose_change: thresholds must be >= 0");
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  unsigned long long* c = reinterpret_cast<unsigned long long*>(counts);
  hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(64), 0, st, c);
  FM_CHECK_LAUNCH(ctx);
  if (s->P == 0) return FM_OK;
  hipLaunchKernelGGL(k_pose_change, dim3(grid_for(s->P, kBlock)), dim3(kBlock), 0, st, params_a, params_b,
                     s->pair_cams, s->P, (double)rot_deg, (double)t_deg, rot_out, t_out, c);
  FM_CHECK_LAUNCH(ctx);
  return FM_OK;
}
