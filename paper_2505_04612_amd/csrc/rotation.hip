// Global rotation averaging (FastMap, arXiv 2505.04612, Sec. 3.3 "Global
// Rotation": eq. rotation-objective with the geodesic distance, the 6D
// rotation parameterisation) on a scene's pair graph.
//
// The per-pair records use the epipolar loop's layout ([P, 24] floats: for
// each side of the pair dL/dR as 3x3 row-major and three unused entries), so
// the camera side shares its row sums and Gram-Schmidt adjoint.  Parameters
// are (a1, a2) per camera, [N, 6].
#include "fm_internal.h"

#include <cmath>

namespace {

__device__ inline double pick3d(const double a[3], int k) { return k == 0 ? a[0] : (k == 1 ? a[1] : a[2]); }

// One pair's geodesic term and its record, float64.  With Q = R^{i->j},
// M = R_j^T Q R_i, c = (tr M - 1)/2 and d = arccos(c) (c clipped to
// [-1, 1]): dd/dc = -1/sqrt(1 - c^2) (0 where |c| = 1), dc/dR_j = Q R_i / 2
// = R_j M / 2 and dc/dR_i = Q^T R_j / 2 = R_i M^T / 2; both scaled by invP.
// The records keep only the part of these that moves along the rotation
// group (R_j K and -R_i K with K = (M - M^T)/2): the rest is annihilated by
// the Gram-Schmidt adjoint, and it grows like 1/d, so a float32 record of
// the full matrix would lose the O(1) tangent part to rounding when d is
// small.  Returns d.
__device__ inline double ra_pair(const double Ri[3][3], const double Rj[3][3], const float* __restrict__ q,
                                 double invP, float* __restrict__ rec) {
  double Q[3][3], QRi[3][3], M[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) Q[a][b] = (double)q[3 * a + b];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) QRi[a][b] = Q[a][0] * Ri[0][b] + Q[a][1] * Ri[1][b] + Q[a][2] * Ri[2][b];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) M[a][b] = Rj[0][a] * QRi[0][b] + Rj[1][a] * QRi[1][b] + Rj[2][a] * QRi[2][b];
  double c = 0.5 * (M[0][0] + M[1][1] + M[2][2] - 1.0);
  const bool inside = c > -1.0 && c < 1.0;
  c = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
  if (rec) {
    const double half_gc = inside ? -0.5 * invP / sqrt(1.0 - c * c) : 0.0;
    double K[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) K[a][b] = 0.5 * (M[a][b] - M[b][a]);
    float gi[12], gj[12];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        gj[3 * a + b] = (float)(half_gc * (Rj[a][0] * K[0][b] + Rj[a][1] * K[1][b] + Rj[a][2] * K[2][b]));
        gi[3 * a + b] = (float)(-half_gc * (Ri[a][0] * K[0][b] + Ri[a][1] * K[1][b] + Ri[a][2] * K[2][b]));
      }
    gi[9] = gi[10] = gi[11] = 0.0f;
    gj[9] = gj[10] = gj[11] = 0.0f;
    float4* dst = reinterpret_cast<float4*>(rec);
    dst[0] = make_float4(gi[0], gi[1], gi[2], gi[3]);
    dst[1] = make_float4(gi[4], gi[5], gi[6], gi[7]);
    dst[2] = make_float4(gi[8], gi[9], gi[10], gi[11]);
    dst[3] = make_float4(gj[0], gj[1], gj[2], gj[3]);
    dst[4] = make_float4(gj[4], gj[5], gj[6], gj[7]);
    dst[5] = make_float4(gj[8], gj[9], gj[10], gj[11]);
  }
  return acos(c);
}

__device__ inline void rot6(const float* __restrict__ p6, int c, double R[3][3]) {
  double a1[3], a2[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    a1[k] = (double)p6[6 * (int64_t)c + k];
    a2[k] = (double)p6[6 * (int64_t)c + 3 + k];
  }
  gs_matrix(gs_forward(a1, a2), R);
}

__device__ inline void load_rot(const double* __restrict__ rot, int c, double R[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) R[a][b] = rot[9 * (int64_t)c + 3 * a + b];
}

// ------------------------------------------------------------------ standalone loss + gradient

__global__ __launch_bounds__(kBlock) void k_ra_pair(const float* __restrict__ params, const int32_t* __restrict__ cams,
                                                    const float* __restrict__ Rrel, int64_t P, double invP,
                                                    float* __restrict__ contrib, double* __restrict__ part) {
  __shared__ double lds[kBlock / 64];
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, gsize = (int64_t)gridDim.x * blockDim.x;
  double v = 0.0;
  for (int64_t n = gtid; n < P; n += gsize) {
    double Ri[3][3], Rj[3][3];
    rot6(params, cams[2 * n], Ri);
    rot6(params, cams[2 * n + 1], Rj);
    v += ra_pair(Ri, Rj, Rrel + 9 * n, invP, contrib + 24 * n);
  }
  const double t = block_sum(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_ra_camera(const float* __restrict__ params,
                                                      const int32_t* __restrict__ cam_ptr,
                                                      const int32_t* __restrict__ cam_items,
                                                      const float* __restrict__ contrib, int32_t N,
                                                      float* __restrict__ grad) {
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = gtid >> 4;
  const int lane = threadIdx.x & 63, l16 = lane & 15;
  if (c >= N) return;   // whole rows leave together: the row exchanges stay within live rows
  double acc[12];
  row_camera_sums(row_list(cam_ptr, cam_items, (int)c, l16), cam_items, contrib, lane, acc);
  double a1[3], a2[3], g[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    a1[k] = (double)params[6 * c + k];
    a2[k] = (double)params[6 * c + 3 + k];
  }
  gs_adjoint(acc, a1, a2, g);
  if (l16 < 6) grad[6 * c + l16] = (float)pick9(g, l16);
}

__global__ void k_ra_loss_final(const double* __restrict__ part, int64_t nblocks, double invP, double* __restrict__ loss) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int64_t b = 0; b < nblocks; ++b) s += part[b];
  *loss = s * invP;
}

// ------------------------------------------------------------------ fused persistent loop

struct RaArgs {
  float* params;
  float* m;
  float* v;
  const int32_t* cams;
  const float* Rrel;
  const int32_t* cam_ptr;
  const int32_t* cam_items;
  float* contrib;
  double* rot;
  double* part;
  double* trace;
  unsigned* bar;
  int64_t P;
  int32_t N;
  int32_t K;
  double invP, lr, log_frac, b1, b2, eps;
  int64_t lr_step0, lr_total, adam_step0;
};

// Rotation of camera c from the parameters p0 held by lanes 0..5 of its row,
// stored by lanes 0..8 (written through to memory if WTS).
template <bool WTS = false>
__device__ inline void ra_store_rot(double* __restrict__ rot, int64_t c, float p0, int base, int l16, bool live) {
  double a1[3], a2[3], R[3][3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    a1[j] = (double)__shfl(p0, base + j);
    a2[j] = (double)__shfl(p0, base + 3 + j);
  }
  if (!live) a1[0] = a2[1] = 1.0;   // a row without a camera: keep Gram-Schmidt away from 0/0
  gs_matrix(gs_forward(a1, a2), R);
  if (live && l16 < 9) {
    double rv = R[0][0];
#pragma unroll
    for (int j = 1; j < 9; ++j) rv = (l16 == j) ? R[j / 3][j % 3] : rv;
    if constexpr (WTS)
      store_wt(&rot[c * 9 + l16], rv);
    else
      rot[c * 9 + l16] = rv;
  }
}

__global__ __launch_bounds__(kSolveBlock) void k_ra_solve(RaArgs a) {
  GridBar gb = grid_bar(a.bar);
  __shared__ double lds[kSolveBlock / 64];
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63;
  const int64_t gwave = gtid >> 6, nwaves = gsize >> 6;
  const int row = lane >> 4, l16 = lane & 15, base = lane & ~15;
  const int64_t c_first = 4 * gwave + row, c_stride = 4 * nwaves;
  // rotations of the initial parameters
  for (int64_t c0 = 4 * gwave; c0 < a.N; c0 += c_stride) {
    const int64_t c = c0 + row;
    const bool live = c < a.N;
    const float p0 = (live && l16 < 6) ? a.params[6 * c + l16] : 0.0f;
    ra_store_rot(a.rot, c, p0, base, l16, live);
  }
  // static data of this thread's first pair and this row's first camera
  int ci0 = 0, cj0 = 0;
  if (gtid < a.P) {
    ci0 = a.cams[2 * gtid];
    cj0 = a.cams[2 * gtid + 1];
  }
  RowList L0 = {0, 0, {-1, -1, -1, -1}};
  if (c_first < a.N) L0 = row_list(a.cam_ptr, a.cam_items, (int)c_first, l16);
  grid_barrier(gb);
  StepSched sch(a.log_frac, a.lr_step0, a.lr_total, a.adam_step0, a.b1, a.b2);
  for (int k = 0; k < a.K; ++k) {
    double v = 0.0;
    for (int64_t n = gtid; n < a.P; n += gsize) {
      double Ri[3][3], Rj[3][3];
      load_rot(a.rot, n == gtid ? ci0 : a.cams[2 * n], Ri);
      load_rot(a.rot, n == gtid ? cj0 : a.cams[2 * n + 1], Rj);
      v += ra_pair(Ri, Rj, a.Rrel + 9 * n, a.invP, a.contrib + 24 * n);
    }
    if (a.trace) {
      const double t = block_sum(v, lds);
      if (threadIdx.x == 0) a.part[blockIdx.x] = t;
    }
    grid_barrier(gb);
    if (a.trace && gtid == 0) {
      double s = 0.0;
      for (int b = 0; b < (int)gridDim.x; ++b) s += a.part[b];
      a.trace[k] = s * a.invP;
    }
    const double lr = a.lr * sch.frac;
    const double bc1 = 1.0 - sch.p1, bc2 = 1.0 - sch.p2;
    sch.next();
    // the loop bound is uniform over the wavefront (rows past N idle), so
    // the row exchanges always run with every lane present
    for (int64_t c0 = 4 * gwave; c0 < a.N; c0 += c_stride) {
      const int64_t c = c0 + row;
      const bool live = c < a.N;
      float p0 = 0.0f, mq = 0.0f, vq = 0.0f;
      if (live && l16 < 6) {
        p0 = a.params[6 * c + l16];
        mq = a.m[6 * c + l16];
        vq = a.v[6 * c + l16];
      }
      double acc[12];
      const RowList L = c0 == 4 * gwave ? L0 : (live ? row_list(a.cam_ptr, a.cam_items, (int)c, l16)
                                                     : RowList{0, 0, {-1, -1, -1, -1}});
      row_camera_sums(L, a.cam_items, a.contrib, lane, acc);
      double a1[3], a2[3], g[9];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        a1[j] = (double)__shfl(p0, base + j);
        a2[j] = (double)__shfl(p0, base + 3 + j);
      }
      if (!live) a1[0] = a2[1] = 1.0;
      gs_adjoint(acc, a1, a2, g);
      float pq = 0.0f;
      if (live && l16 < 6) {
        pq = adam_update(p0, (float)pick9(g, l16), mq, vq, lr, a.b1, a.b2, a.eps, bc1, bc2);
        a.params[6 * c + l16] = pq;
        a.m[6 * c + l16] = mq;
        a.v[6 * c + l16] = vq;
      }
      ra_store_rot(a.rot, c, pq, base, l16, live);
    }
    grid_barrier(gb);
  }
}

// Camera-by-camera variant of the loop (the automatic choice): one
// wavefront per camera; each lane evaluates one
// of the camera's pairs and keeps its own side of the record (float32, as
// the records are), the wavefront sums them in a fixed order and lanes 0..5
// take the Adam steps.  No records are exchanged, so an iteration needs one
// grid barrier; the parameters and rotations other wavefronts read are
// double-buffered by iteration parity.
struct RaCamArgs {
  float* params;       // buffer 0 [N, 6] (the caller's)
  float* alt;          // buffer 1 [N, 6]
  float* m;
  float* v;
  const int32_t* cams;
  const float* Rrel;
  const int32_t* cam_ptr;
  const int32_t* cam_items;
  double* rot;         // [2, N, 9]
  double* part;        // [2, gridDim.x]
  double* trace;
  unsigned* bar;
  int64_t P;
  int32_t N;
  int32_t K;
  double invP, lr, log_frac, b1, b2, eps;
  int64_t lr_step0, lr_total, adam_step0;
};

// Static data of one incidence entry: the entry (pair << 1 | side), both
// cameras and the pair's relative rotation.
struct RaEntry {
  int item, ci, cj;
  float q[9];
};

__device__ inline RaEntry ra_entry(const RaCamArgs& a, int q) {
  RaEntry e;
  e.item = a.cam_items[q];
  const int64_t n = e.item >> 1;
  e.ci = a.cams[2 * n];
  e.cj = a.cams[2 * n + 1];
#pragma unroll
  for (int k = 0; k < 9; ++k) e.q[k] = a.Rrel[9 * n + k];
  return e;
}

__global__ __launch_bounds__(kSolveBlock) void k_ra_solve_cam(RaCamArgs a) {
  GridBar gb = grid_bar(a.bar);
  __shared__ double lds[kSolveBlock / 64];
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63;
  const int64_t gwave = gtid >> 6, nwaves = gsize >> 6;
  const int kq = lane < 6 ? lane : 5;
  const int64_t NR = (int64_t)a.N * 9;
  // rotations of the initial parameters (buffer 0)
  for (int64_t c = gwave; c < a.N; c += nwaves) ra_store_rot(a.rot, c, a.params[6 * c + kq], 0, lane, true);
  grid_barrier(gb);
  // static data of the first 64 incidence entries of this wavefront's first
  // camera (one per lane), read once for the launch
  RaEntry e0{};
  if (gwave < a.N) {
    const int lo = a.cam_ptr[gwave], hi = a.cam_ptr[gwave + 1];
    if (lo + lane < hi) e0 = ra_entry(a, lo + lane);
  }
  StepSched sch(a.log_frac, a.lr_step0, a.lr_total, a.adam_step0, a.b1, a.b2);
  for (int k = 0; k < a.K; ++k) {
    const int rb = k & 1;
    const float* pr = rb ? a.alt : a.params;
    float* pw = rb ? a.params : a.alt;
    const double* rr = a.rot + rb * NR;
    double* rw = a.rot + (rb ^ 1) * NR;
    const double lr = a.lr * sch.frac;
    const double bc1 = 1.0 - sch.p1, bc2 = 1.0 - sch.p2;
    sch.next();
    double lsum = 0.0;
    // the loop bound is uniform over the wavefront, so the wavefront sums
    // run with every lane present
    for (int64_t c = gwave; c < a.N; c += nwaves) {
      const int lo = a.cam_ptr[c], hi = a.cam_ptr[c + 1];
      const float p0 = pr[6 * c + kq];
      float mq = a.m[6 * c + kq], vq = a.v[6 * c + kq];
      double acc[12];
#pragma unroll
      for (int j = 0; j < 12; ++j) acc[j] = 0.0;
      for (int q = lo + lane; q < hi; q += 64) {
        // the lane's first entry of the wavefront's first camera from
        // registers (read once per launch), the others from memory
        RaEntry e;
        if (c == gwave && q == lo + lane)
          e = e0;
        else
          e = ra_entry(a, q);
        const int side = e.item & 1;
        double Ri[3][3], Rj[3][3];
        load_rot(rr, e.ci, Ri);
        load_rot(rr, e.cj, Rj);
        float rec[24];
        const double d = ra_pair(Ri, Rj, e.q, a.invP, rec);
        if (side == 0) lsum += d;   // each pair's term once, from its first camera
#pragma unroll
        for (int j = 0; j < 12; ++j) acc[j] += (double)(side ? rec[12 + j] : rec[j]);
      }
      wave_sum12(acc, lane);
      double a1[3], a2[3], g[9];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        a1[j] = (double)__shfl(p0, j);
        a2[j] = (double)__shfl(p0, 3 + j);
      }
      gs_adjoint(acc, a1, a2, g);
      const float pq = adam_update(p0, (float)pick9(g, kq), mq, vq, lr, a.b1, a.b2, a.eps, bc1, bc2);
      // parameters, rotations and loss partials are read by other
      // workgroups after the barrier: written through to memory
      if (lane < 6) {
        store_wt(&pw[6 * c + lane], pq);
        a.m[6 * c + lane] = mq;
        a.v[6 * c + lane] = vq;
      }
      ra_store_rot<true>(rw, c, pq, 0, lane, true);
    }
    if (a.trace) {
      const double t = block_sum(lsum, lds);
      if (threadIdx.x == 0) store_wt(&a.part[rb * gridDim.x + blockIdx.x], t);
    }
    grid_barrier_wt(gb);
    if (a.trace && gtid == 0) {
      double t = 0.0;
      for (int b = 0; b < (int)gridDim.x; ++b) t += a.part[rb * gridDim.x + b];
      a.trace[k] = t * a.invP;
    }
  }
  // after an odd number of iterations the latest parameters are in buffer 1
  if (a.K & 1) {
    for (int64_t c = gwave; c < a.N; c += nwaves)
      if (lane < 6) a.params[6 * c + lane] = a.alt[6 * c + lane];
  }
}

// ------------------------------------------------------------------ initialisation (column-wise least squares)

// The quadratic forms of the appendix on rotation initialisation, as an
// operator on stacked 3-vectors v [N,3]:
//   (A v)_c = sum over pairs n = (i, j) containing c of
//             v_j - Q v_i          (c = j),
//             Q^T Q v_i - Q^T v_j  (c = i),
// which is x^T A x = sum_n |x_j - Q x_i|^2; the second-column problem uses
// alpha A + beta diag(u_c u_c^T) with alpha = 1/P, beta = 1/N and u the
// first columns.  The smallest eigenvector comes from Lanczos with full
// (twice applied) classical Gram-Schmidt reorthogonalisation, the smallest
// eigenpair of the tridiagonal matrix (Sturm bisection, inverse iteration)
// and the Ritz vector.

struct LzArgs {
  const int32_t* cams;
  const float* Rrel;
  const int32_t* cam_ptr;
  const int32_t* cam_items;
  const double* start;   // [n]
  const double* u;       // [n] or null (first columns for the second problem)
  double* V;             // [m + 1, n]
  double* w;             // [n]
  double* h;             // [m + 1] dots of the current step
  double* part;          // [waves] partial sums
  double* alpha;         // [m]
  double* beta;          // [m]
  double* s;             // [m] Ritz coefficients; also [3m] scratch after it
  double* out;           // [n] Ritz vector
  double* info;          // [2]: Ritz value, steps taken
  unsigned* bar;
  int64_t n;
  int32_t N;
  int32_t m;
  double op_alpha, op_beta;
};

// Sum over the grid of one double per thread, returned in every thread
// (per-wavefront sums, then every workgroup adds them in the same order).
__device__ inline double grid_allsum(double v, double* part, double* lds1, GridBar& gb, int64_t gwave, int64_t nwaves) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s);
  if ((threadIdx.x & 63) == 0) part[gwave] = v;
  grid_barrier(gb);
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int64_t k = 0; k < nwaves; ++k) t += part[k];
    lds1[0] = t;
  }
  __syncthreads();
  const double t = lds1[0];
  __syncthreads();
  return t;
}

// y = op(v) for camera c in every lane of its 16-lane row.
__device__ inline void lz_apply(const LzArgs& a, const double* __restrict__ v, int64_t c, int l16, double y[3]) {
  y[0] = y[1] = y[2] = 0.0;
  const int lo = a.cam_ptr[c], hi = a.cam_ptr[c + 1];
  double vc[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) vc[k] = v[3 * c + k];
  for (int q = lo + l16; q < hi; q += 16) {
    const int item = a.cam_items[q];
    const int64_t n = item >> 1;
    const bool is_j = item & 1;
    const int other = a.cams[2 * n + (is_j ? 0 : 1)];
    double Q[3][3], vo[3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k) Q[r][k] = (double)a.Rrel[9 * n + 3 * r + k];
#pragma unroll
    for (int k = 0; k < 3; ++k) vo[k] = v[3 * (int64_t)other + k];
    if (is_j) {
      // v_j - Q v_i
#pragma unroll
      for (int r = 0; r < 3; ++r) y[r] += vc[r] - (Q[r][0] * vo[0] + Q[r][1] * vo[1] + Q[r][2] * vo[2]);
    } else {
      // Q^T (Q v_i - v_j)
      double t[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) t[r] = Q[r][0] * vc[0] + Q[r][1] * vc[1] + Q[r][2] * vc[2] - vo[r];
#pragma unroll
      for (int k = 0; k < 3; ++k) y[k] += Q[0][k] * t[0] + Q[1][k] * t[1] + Q[2][k] * t[2];
    }
  }
#pragma unroll
  for (int s = 8; s >= 1; s >>= 1)
#pragma unroll
    for (int k = 0; k < 3; ++k) y[k] += __shfl_xor(y[k], s);
#pragma unroll
  for (int k = 0; k < 3; ++k) y[k] *= a.op_alpha;
  if (a.u) {
    double uc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) uc[k] = a.u[3 * c + k];
    const double d = uc[0] * vc[0] + uc[1] * vc[1] + uc[2] * vc[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) y[k] += a.op_beta * uc[k] * d;
  }
}

// Number of eigenvalues of the symmetric tridiagonal (alpha, beta) below x
// (Sturm sequence of the LDL^T pivots).
__device__ inline int sturm_count(const double* alpha, const double* beta, int m, double x) {
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < m; ++i) {
    const double b2 = i > 0 ? beta[i - 1] * beta[i - 1] : 0.0;
    d = alpha[i] - x - (i > 0 ? b2 / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) ++cnt;
  }
  return cnt;
}

// Smallest eigenpair of the m x m symmetric tridiagonal matrix (one thread):
// bisection on the Sturm count, then inverse iteration with a pivoted
// tridiagonal solve.  s [m] receives the unit eigenvector; scratch [3m].
__device__ inline double tridiag_smallest(const double* alpha, const double* beta, int m, double* s, double* scratch) {
  double lo = alpha[0], hi = alpha[0];
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? fabs(beta[i - 1]) : 0.0) + (i + 1 < m ? fabs(beta[i]) : 0.0);
    lo = fmin(lo, alpha[i] - r);
    hi = fmax(hi, alpha[i] + r);
  }
  for (int it = 0; it < 200 && hi - lo > 1e-15 * fmax(1.0, fabs(lo) + fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_count(alpha, beta, m, mid) >= 1) hi = mid;
    else lo = mid;
  }
  const double theta = 0.5 * (lo + hi);
  const double sigma = theta - 1e-10 * fmax(1.0, fabs(theta));
  // (T - sigma I) z = s by Gaussian elimination with partial pivoting
  // (rows i and i+1 may swap; the factors have up to two superdiagonals)
  double* u1 = scratch;          // first superdiagonal of U
  double* u2 = scratch + m;      // second superdiagonal of U
  double* dd = scratch + 2 * m;  // diagonal of U
  for (int i = 0; i < m; ++i) s[i] = 1.0;
  for (int iter = 0; iter < 3; ++iter) {
    // factor and solve in one sweep: row i holds (dd[i], u1[i], u2[i])
    double* rhs = s;
    double cur_d = alpha[0] - sigma, cur_u1 = m > 1 ? beta[0] : 0.0, cur_u2 = 0.0;
    double cur_r = rhs[0];
    for (int i = 0; i < m; ++i) {
      if (i + 1 < m) {
        const double nb = beta[i];                         // sub-diagonal entry of row i+1
        const double nd = alpha[i + 1] - sigma, nu1 = i + 2 < m ? beta[i + 1] : 0.0;
        const double nr = rhs[i + 1];
        if (fabs(cur_d) >= fabs(nb)) {
          const double l = nb / (cur_d != 0.0 ? cur_d : 1e-300);
          dd[i] = cur_d; u1[i] = cur_u1; u2[i] = cur_u2; rhs[i] = cur_r;
          cur_d = nd - l * cur_u1;
          cur_u1 = nu1 - l * cur_u2;
          cur_u2 = 0.0;
          cur_r = nr - l * cur_r;
        } else {
          const double l = cur_d / nb;
          dd[i] = nb; u1[i] = nd; u2[i] = nu1; rhs[i] = nr;
          const double od = cur_d, ou1 = cur_u1, ou2 = cur_u2, orr = cur_r;
          (void)od;
          cur_d = ou1 - l * nd;
          cur_u1 = ou2 - l * nu1;
          cur_u2 = 0.0;
          cur_r = orr - l * nr;
        }
      } else {
        dd[i] = cur_d != 0.0 ? cur_d : 1e-300; u1[i] = 0.0; u2[i] = 0.0; rhs[i] = cur_r;
      }
    }
    for (int i = m - 1; i >= 0; --i) {
      double t = rhs[i];
      if (i + 1 < m) t -= u1[i] * s[i + 1];
      if (i + 2 < m) t -= u2[i] * s[i + 2];
      s[i] = t / (dd[i] != 0.0 ? dd[i] : 1e-300);
    }
    double nrm = 0.0;
    for (int i = 0; i < m; ++i) nrm += s[i] * s[i];
    nrm = 1.0 / sqrt(nrm);
    for (int i = 0; i < m; ++i) s[i] *= nrm;
  }
  return theta;
}

// Lanczos steps between convergence checks, and the relative residual
// bound |beta_k s_k| / |T| below which the Ritz pair is taken as converged.
constexpr int kLzCheck = 10;
constexpr int kLzMaxSteps = 4096;
constexpr double kLzTol = 1e-11;

__global__ __launch_bounds__(kSolveBlock) void k_ra_lanczos(LzArgs a) {
  GridBar gb = grid_bar(a.bar);
  extern __shared__ double hs[];   // [m + 1] dots of the current step, then [1] broadcast
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63;
  const int64_t gwave = gtid >> 6, nwaves = gsize >> 6;
  const int row = lane >> 4, l16 = lane & 15;
  const int64_t n = a.n;
  double* lds1 = hs + a.m + 1;
  // q0 = start / |start|
  double acc = 0.0;
  for (int64_t i = gtid; i < n; i += gsize) acc += a.start[i] * a.start[i];
  const double inv0 = 1.0 / sqrt(grid_allsum(acc, a.part, lds1, gb, gwave, nwaves));
  for (int64_t i = gtid; i < n; i += gsize) a.V[i] = a.start[i] * inv0;
  grid_barrier(gb);
  int m = a.m;
  bool have_s = false;
  for (int k = 0; k < a.m; ++k) {
    const double* q = a.V + (int64_t)k * n;
    // w = op(q_k)
    for (int64_t c0 = 4 * gwave; c0 < a.N; c0 += 4 * nwaves) {
      const int64_t c = c0 + row;
      if (c < a.N) {   // whole rows: the row exchanges stay within live rows
        double y[3];
        lz_apply(a, q, c, l16, y);
        if (l16 < 3) a.w[3 * c + l16] = pick3d(y, l16);
      }
    }
    grid_barrier(gb);
    // two passes of classical Gram-Schmidt against q_0 .. q_k
    double alpha_k = 0.0;
    bool stop = false;
    for (int pass = 0; pass < 2; ++pass) {
      for (int64_t j = gwave; j <= k; j += nwaves) {
        const double* vj = a.V + j * n;
        double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
        int64_t i = lane;
        for (; i + 192 < n; i += 256) {
          d0 += vj[i] * a.w[i];
          d1 += vj[i + 64] * a.w[i + 64];
          d2 += vj[i + 128] * a.w[i + 128];
          d3 += vj[i + 192] * a.w[i + 192];
        }
        for (; i < n; i += 64) d0 += vj[i] * a.w[i];
        double d = (d0 + d1) + (d2 + d3);
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) d += __shfl_xor(d, s);
        if (lane == 0) a.h[j] = d;
      }
      grid_barrier(gb);
      for (int j = threadIdx.x; j <= k; j += blockDim.x) hs[j] = a.h[j];
      __syncthreads();
      alpha_k += hs[k];
      // w_i -= sum_j h_j V[j][i], eight basis entries in flight per thread
      double nrm = 0.0;
      for (int64_t i = gtid; i < n; i += gsize) {
        double s8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int j = 0;
        for (; j + 8 <= k + 1; j += 8) {
          double v8[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v8[u] = a.V[(int64_t)(j + u) * n + i];
#pragma unroll
          for (int u = 0; u < 8; ++u) s8[u] += hs[j + u] * v8[u];
        }
        for (; j <= k; ++j) s8[0] += hs[j] * a.V[(int64_t)j * n + i];
        const double wi = a.w[i] - (((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7])));
        a.w[i] = wi;
        nrm += wi * wi;
      }
      __syncthreads();   // hs is rewritten by the next pass
      if (pass == 0) {
        grid_barrier(gb);
      } else {
        const double b = sqrt(grid_allsum(nrm, a.part, lds1, gb, gwave, nwaves));
        if (gtid == 0) {
          a.alpha[k] = alpha_k;
          a.beta[k] = b;
        }
        // an invariant subspace, the last step, or a converged Ritz pair
        // (checked every kLzCheck steps by one thread; the decision is read
        // by all after a barrier)
        if (!(b > 1e-12 * fmax(1.0, fabs(alpha_k))) || k + 1 == a.m) {
          stop = true;
        } else if ((k + 1) % kLzCheck == 0) {
          grid_barrier(gb);   // alpha, beta of this step visible
          if (gtid == 0) {
            const double theta = tridiag_smallest(a.alpha, a.beta, k + 1, a.s, a.s + a.m);
            double tn = 0.0;
            for (int i = 0; i <= k; ++i) tn = fmax(tn, fabs(a.alpha[i]) + 2.0 * fabs(a.beta[i]));
            a.info[0] = theta;
            a.h[a.m] = (fabs(b * a.s[k]) <= kLzTol * fmax(tn, 1e-300)) ? 1.0 : 0.0;
          }
          grid_barrier(gb);
          stop = a.h[a.m] != 0.0;
          have_s = stop;
        }
        if (stop) {
          m = k + 1;
        } else {
          const double inv = 1.0 / b;
          double* qn = a.V + (int64_t)(k + 1) * n;
          for (int64_t i = gtid; i < n; i += gsize) qn[i] = a.w[i] * inv;
        }
      }
    }
    if (stop) break;
    grid_barrier(gb);
  }
  grid_barrier(gb);
  if (gtid == 0) {
    if (!have_s) a.info[0] = tridiag_smallest(a.alpha, a.beta, m, a.s, a.s + a.m);
    a.info[1] = (double)m;
  }
  grid_barrier(gb);
  for (int64_t i = gtid; i < n; i += gsize) {
    double x = 0.0;
    for (int j = 0; j < m; ++j) x += a.s[j] * a.V[(int64_t)j * n + i];
    a.out[i] = x;
  }
}

// c1 = x_c / |x_c| per camera (first columns); also copied to u for the
// second problem.
__global__ __launch_bounds__(kBlock) void k_ra_unit_rows(const double* __restrict__ x, int32_t N, double* __restrict__ u) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const double a = x[3 * c], b = x[3 * c + 1], d = x[3 * c + 2];
  const double r = 1.0 / sqrt(a * a + b * b + d * d);
  u[3 * c] = a * r;
  u[3 * c + 1] = b * r;
  u[3 * c + 2] = d * r;
}

// Second columns: y_c normalised, made orthogonal to c1 (Gram-Schmidt) and
// normalised again; the parameters are (c1, c2), the rotation's first two
// columns (its third is c1 x c2 by the 6D map).
__global__ __launch_bounds__(kBlock) void k_ra_finish(const double* __restrict__ c1, const double* __restrict__ y,
                                                      int32_t N, float* __restrict__ params) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  double v[3], e[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v[k] = y[3 * c + k];
    e[k] = c1[3 * c + k];
  }
  double r = 1.0 / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
#pragma unroll
  for (int k = 0; k < 3; ++k) v[k] *= r;
  const double d = v[0] * e[0] + v[1] * e[1] + v[2] * e[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) v[k] -= d * e[k];
  r = 1.0 / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    params[6 * c + k] = (float)e[k];
    params[6 * c + 3 + k] = (float)(v[k] * r);
  }
}

fm_status ra_check(fm_ctx* ctx, fm_scene* s, const char* fn) {
  if (!s) return fm_fail(ctx, FM_EINVAL, "%s: scene is NULL", fn);
  if (s->ctx != ctx) return fm_fail(ctx, FM_EINVAL, "%s: scene belongs to another context", fn);
  return FM_OK;
}

}  // namespace

extern "C" fm_status fm_rotation_loss_grad(fm_ctx* ctx, fm_scene* s, const float* Rrel, const float* params,
                                           double* loss, float* grad, fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  fm_status rc = ra_check(ctx, s, "fm_rotation_loss_grad");
  if (rc != FM_OK) return rc;
  if ((s->P > 0 && !Rrel) || (s->N > 0 && !params)) return fm_fail(ctx, FM_EINVAL, "fm_rotation_loss_grad: NULL argument");
  if (!loss && !grad) return FM_OK;
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const double invP = s->P > 0 ? 1.0 / (double)s->P : 0.0;
  const unsigned gp = grid_for(s->P > 0 ? s->P : 1, kBlock);
  {
    fm_timed timer(ctx, FM_K_RA_PAIR, st);
    hipLaunchKernelGGL(k_ra_pair, dim3(gp), dim3(kBlock), 0, st, params, s->pair_cams, Rrel, s->P, invP, s->contrib,
                       s->loss_part);
    FM_CHECK_LAUNCH(ctx);
  }
  if (loss) {
    hipLaunchKernelGGL(k_ra_loss_final, dim3(1), dim3(64), 0, st, s->loss_part, (int64_t)gp, invP, loss);
    FM_CHECK_LAUNCH(ctx);
  }
  if (grad && s->N > 0) {
    fm_timed timer(ctx, FM_K_RA_CAMERA, st);
    hipLaunchKernelGGL(k_ra_camera, dim3(grid_for((int64_t)s->N * 16, kBlock)), dim3(kBlock), 0, st, params,
                       s->cam_ptr, s->cam_items, s->contrib, s->N, grad);
    FM_CHECK_LAUNCH(ctx);
  }
  return FM_OK;
}

extern "C" fm_status fm_rotation_solve(fm_ctx* ctx, fm_scene* s, const float* Rrel, float* params, float* m, float* v,
                                       int32_t K, const fm_adam_cfg* cfg, double* loss_trace, fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  fm_status rc = ra_check(ctx, s, "fm_rotation_solve");
  if (rc != FM_OK) return rc;
  if (!cfg || (s->P > 0 && !Rrel) || (s->N > 0 && (!params || !m || !v)))
    return fm_fail(ctx, FM_EINVAL, "fm_rotation_solve: NULL argument");
  if (K < 0) return fm_fail(ctx, FM_EINVAL, "fm_rotation_solve: K < 0");
  if (cfg->lr_total_steps <= 0 || cfg->lr_step0 < 0 || cfg->adam_step0 < 0 || !(cfg->lr_final_frac > 0.0f) ||
      !(cfg->lr_rot >= 0.0f) ||
      !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f && cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f && cfg->eps >= 0.0f))
    return fm_fail(ctx, FM_EINVAL, "fm_rotation_solve: bad Adam configuration");
  if (K == 0 || s->N == 0) return FM_OK;
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  if (s->ra_coop_blocks <= 0) {
    int per_cu = 0;
    FM_HIP_TRY(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ra_solve, kSolveBlock, 0));
    int per_cu_cam = 0;
    FM_HIP_TRY(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_cam, k_ra_solve_cam, kSolveBlock, 0));
    if (per_cu_cam < per_cu) per_cu = per_cu_cam;
    s->ra_coop_blocks = per_cu * ctx->num_cu;
    if (s->ra_coop_blocks <= 0) return fm_fail(ctx, FM_ECOOP, "cannot size the cooperative rotation kernel");
  }
  // sized like the epipolar loop
  int64_t want = grid_for(s->P, kSolveBlock);
  const int64_t want_c = grid_for((int64_t)s->N * 16, kSolveBlock);
  if (want_c > want) want = want_c;
  if (want > (s->P < 32768 ? 16 : 192)) want = s->P < 32768 ? 16 : 192;
  if (cfg->blocks > 0) want = cfg->blocks;
  if (want < 1) want = 1;
  if (want > s->ra_coop_blocks) want = s->ra_coop_blocks;
  if (want > s->loss_part_cap) want = s->loss_part_cap;
  RaArgs a;
  a.params = params; a.m = m; a.v = v;
  a.cams = s->pair_cams; a.Rrel = Rrel; a.cam_ptr = s->cam_ptr; a.cam_items = s->cam_items;
  a.contrib = s->contrib; a.rot = s->rot; a.part = s->loss_part; a.trace = loss_trace; a.bar = s->bar;
  a.P = s->P; a.N = s->N; a.K = K;
  a.invP = s->P > 0 ? 1.0 / (double)s->P : 0.0;
  a.lr = cfg->lr_rot; a.log_frac = log((double)cfg->lr_final_frac);
  a.b1 = cfg->beta1; a.b2 = cfg->beta2; a.eps = cfg->eps;
  a.lr_step0 = cfg->lr_step0; a.lr_total = cfg->lr_total_steps; a.adam_step0 = cfg->adam_step0;
  void* args[] = {&a};
  FM_HIP_TRY(ctx, fm_bar_reset(s->bar, st));
  // automatic grid: the camera loop, one wavefront per camera up to the
  // co-resident limit (faster at every size measured, up to the 5,000-camera
  // street graph with 185k pairs: 26.3 against 36.1 us per iteration)
  const CamGrid cg = cam_grid(s->N, s->ra_coop_blocks, ctx->num_cu);
  const int64_t want_cam = cg.blocks;
  if (cfg->blocks <= 0 && 2 * want_cam <= s->loss_part_cap) {
    RaCamArgs ca;
    ca.params = params; ca.alt = s->params_alt; ca.m = m; ca.v = v;
    ca.cams = s->pair_cams; ca.Rrel = Rrel; ca.cam_ptr = s->cam_ptr; ca.cam_items = s->cam_items;
    ca.rot = s->rot; ca.part = s->loss_part; ca.trace = loss_trace; ca.bar = s->bar;
    ca.P = s->P; ca.N = s->N; ca.K = K;
    ca.invP = a.invP; ca.lr = a.lr; ca.log_frac = a.log_frac; ca.b1 = a.b1; ca.b2 = a.b2; ca.eps = a.eps;
    ca.lr_step0 = a.lr_step0; ca.lr_total = a.lr_total; ca.adam_step0 = a.adam_step0;
    void* cargs[] = {&ca};
    fm_timed timer(ctx, FM_K_RA_SOLVE, st);
    hipError_t e = hipLaunchCooperativeKernel((const void*)k_ra_solve_cam, dim3((unsigned)want_cam),
                                              dim3(cg.threads), cargs, 0, st);
    if (e != hipSuccess) return fm_fail(ctx, FM_ECOOP, "cooperative launch failed: %s", hipGetErrorString(e));
    return FM_OK;
  }
  fm_timed timer(ctx, FM_K_RA_SOLVE, st);
  hipError_t e = hipLaunchCooperativeKernel((const void*)k_ra_solve, dim3((unsigned)want), dim3(kSolveBlock), args, 0, st);
  if (e != hipSuccess) return fm_fail(ctx, FM_ECOOP, "cooperative launch failed: %s", hipGetErrorString(e));
  return FM_OK;
}

extern "C" fm_status fm_rotation_init(fm_ctx* ctx, fm_scene* s, const float* Rrel, const double* start,
                                      int32_t steps, int32_t blocks, float* params, double* info, fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  fm_status rc = ra_check(ctx, s, "fm_rotation_init");
  if (rc != FM_OK) return rc;
  if (s->N == 0) return FM_OK;
  if (!start || !params || (s->P > 0 && !Rrel)) return fm_fail(ctx, FM_EINVAL, "fm_rotation_init: NULL argument");
  if (steps < 1) return fm_fail(ctx, FM_EINVAL, "fm_rotation_init: steps must be >= 1");
  if (blocks < 0) return fm_fail(ctx, FM_EINVAL, "fm_rotation_init: blocks < 0");
  if (s->P == 0) return fm_fail(ctx, FM_ESHAPE, "fm_rotation_init: the pair graph is empty");
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = 3 * (int64_t)s->N;
  const int32_t m = steps < n ? steps : (int32_t)n;
  if (m > kLzMaxSteps) return fm_fail(ctx, FM_EINVAL, "fm_rotation_init: steps above %d", kLzMaxSteps);
  const size_t lds_bytes = sizeof(double) * (kLzMaxSteps + 2);
  if (s->lz_coop_blocks <= 0) {
    int per_cu = 0;
    FM_HIP_TRY(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ra_lanczos, kSolveBlock, lds_bytes));
    s->lz_coop_blocks = per_cu * ctx->num_cu;
    if (s->lz_coop_blocks <= 0) return fm_fail(ctx, FM_ECOOP, "cannot size the cooperative Lanczos kernel");
  }
  // about one 16-lane row per camera, at most 16 workgroups (the solve is a
  // chain of grid-wide reductions), at the co-resident limit
  int64_t want = grid_for(n / 3 * 16, kSolveBlock);
  if (want > 16) want = 16;
  if (blocks > 0) want = blocks;
  if (want < 1) want = 1;
  if (want > s->lz_coop_blocks) want = s->lz_coop_blocks;
  const int64_t waves = want * (kSolveBlock / 64);
  // layout: V [(m+1) n] | w [n] | out [n] | c1 [n] | y [n] | h [m+2] | part [waves] | alpha [m] | beta [m] |
  //         s [4m] | info [4]  (h [m+2]: the last slot carries the convergence decision)
  const int64_t need = (int64_t)(m + 1) * n + 4 * n + (m + 2) + waves + 2 * (int64_t)m + 4 * (int64_t)m + 4;
  if (need > s->lz_cap) {
    FM_HIP_TRY(ctx, hipDeviceSynchronize());
    (void)hipFree(s->lz);
    s->lz = nullptr;
    s->lz_cap = 0;
    if (hipMalloc(&s->lz, sizeof(double) * need) != hipSuccess) {
      (void)hipGetLastError();
      return fm_fail(ctx, FM_ENOMEM, "fm_rotation_init: workspace of %lld doubles", (long long)need);
    }
    s->lz_cap = need;
  }
  double* V = s->lz;
  double* w = V + (int64_t)(m + 1) * n;
  double* out = w + n;
  double* c1 = out + n;
  double* y = c1 + n;
  double* h = y + n;
  double* part = h + (m + 2);
  double* alpha = part + waves;
  double* beta = alpha + m;
  double* sv = beta + m;
  double* inf = sv + 4 * (int64_t)m;
  LzArgs a;
  a.cams = s->pair_cams; a.Rrel = Rrel; a.cam_ptr = s->cam_ptr; a.cam_items = s->cam_items;
  a.V = V; a.w = w; a.h = h; a.part = part; a.alpha = alpha; a.beta = beta; a.s = sv; a.bar = s->bar;
  a.n = n; a.N = s->N; a.m = m;
  fm_timed timer(ctx, FM_K_RA_INIT, st);
  for (int col = 0; col < 2; ++col) {
    a.start = start + col * n;
    a.u = col == 0 ? nullptr : c1;
    a.op_alpha = col == 0 ? 1.0 : 1.0 / (double)s->P;
    a.op_beta = col == 0 ? 0.0 : 1.0 / (double)s->N;
    a.out = col == 0 ? out : y;
    a.info = inf + 2 * col;
    void* args[] = {&a};
    FM_HIP_TRY(ctx, fm_bar_reset(s->bar, st));
    hipError_t e = hipLaunchCooperativeKernel((const void*)k_ra_lanczos, dim3((unsigned)want), dim3(kSolveBlock), args,
                                              lds_bytes, st);
    if (e != hipSuccess) return fm_fail(ctx, FM_ECOOP, "cooperative launch failed: %s", hipGetErrorString(e));
    if (col == 0) {
      hipLaunchKernelGGL(k_ra_unit_rows, dim3(grid_for(s->N, kBlock)), dim3(kBlock), 0, st, out, s->N, c1);
      FM_CHECK_LAUNCH(ctx);
    }
  }
  hipLaunchKernelGGL(k_ra_finish, dim3(grid_for(s->N, kBlock)), dim3(kBlock), 0, st, c1, y, s->N, params);
  FM_CHECK_LAUNCH(ctx);
  if (info) FM_HIP_TRY(ctx, hipMemcpyAsync(info, inf, sizeof(double) * 4, hipMemcpyDeviceToDevice, st));
  return FM_OK;
}
