// Global translation averaging (FastMap, arXiv 2505.04612, Sec. 3.3 "Global
// Translation", eq. global-translation-objective; App. "Multiple
// Initializations") on a scene's pair graph.
//
// Independent runs share every launch: centres and Adam moments are laid out
// [runs, N, 3] and the per-pair records [runs, P] (float4: dL/ds and the
// pair's L1 term), so a thread loads its pair's cameras and target once and
// evaluates the pair for every run, and a 16-lane row reads its camera's
// incidence list once and sums it for every run.  Every sum over a camera's
// pairs runs in the same lane order whatever the grid, so the centres a solve
// produces do not depend on the launch shape.
#include "fm_internal.h"

#include <cmath>

namespace {

constexpr int kTaMaxRuns = 64;

// The L1 term of eq. global-translation-objective for one pair, float64, from
// s = o_j - o_i: u = s/|s|, |u - d|_1.  With `g` it also writes
// dL/ds = (I - u u^T) sign(u - d) * invP / |s| (sign(0) = 0).  A pair whose
// centres coincide has no direction: term and record are 0.
__device__ inline double ta_term(const double s[3], const double d[3], double invP, double* g) {
  const double ns = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
  if (!(ns > 0.0)) {
    if (g) g[0] = g[1] = g[2] = 0.0;
    return 0.0;
  }
  const double r = 1.0 / ns;
  double u[3], sg[3], term = 0.0, ug = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    u[k] = s[k] * r;
    const double e = u[k] - d[k];
    term += fabs(e);
    sg[k] = e > 0.0 ? invP : (e < 0.0 ? -invP : 0.0);
    ug += u[k] * sg[k];
  }
  if (g) {
#pragma unroll
    for (int k = 0; k < 3; ++k) g[k] = (sg[k] - u[k] * ug) * r;
  }
  return term;
}

__device__ inline double ta_term_at(const float* __restrict__ oi, const float* __restrict__ oj, const double d[3]) {
  double s[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) s[k] = (double)oj[k] - (double)oi[k];
  return ta_term(s, d, 0.0, nullptr);
}

// Runs are taken in groups of kTaGroup (the rest in a group of two and a
// single run): every load a group needs is issued, unconditionally, before any of its arithmetic, so a
// thread waits for memory once per group rather than once per run.  (A load
// under a lane condition makes the compiler wait for it on its own.)
constexpr int kTaGroup = 4;

__device__ inline void load_dir(const float* __restrict__ dirs, int64_t n, double d[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) d[k] = (double)dirs[3 * n + k];
}

// One pair for runs r0 .. r0 + G - 1: records [runs, P].
template <int G>
__device__ inline void ta_pair_group(const float* __restrict__ centres, int64_t run_stride, int r0, int64_t P,
                                     int64_t n, int ci, int cj, const double d[3], double invP,
                                     float4* __restrict__ rec) {
  float oi[G][3], oj[G][3];
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const float* o = centres + (r0 + q) * run_stride;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      oi[q][k] = o[3 * (int64_t)ci + k];
      oj[q][k] = o[3 * (int64_t)cj + k];
    }
  }
#pragma unroll
  for (int q = 0; q < G; ++q) {
    double sv[3], g[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) sv[k] = (double)oj[q][k] - (double)oi[q][k];
    const double term = ta_term(sv, d, invP, g);
    rec[(r0 + q) * P + n] = make_float4((float)g[0], (float)g[1], (float)g[2], (float)term);
  }
}

__device__ inline void ta_pair_runs(const float* __restrict__ centres, int32_t N, int runs, int64_t P, int64_t n,
                                    int ci, int cj, const double d[3], double invP, float4* __restrict__ rec) {
  const int64_t run_stride = (int64_t)N * 3;
  int r0 = 0;
  for (; r0 + kTaGroup <= runs; r0 += kTaGroup) ta_pair_group<kTaGroup>(centres, run_stride, r0, P, n, ci, cj, d, invP, rec);
  if (r0 + 2 <= runs) {
    ta_pair_group<2>(centres, run_stride, r0, P, n, ci, cj, d, invP, rec);
    r0 += 2;
  }
  if (r0 < runs) ta_pair_group<1>(centres, run_stride, r0, P, n, ci, cj, d, invP, rec);
}

// Per-run workgroup sums of the pair terms this workgroup's threads wrote
// (each thread re-reads its own records): part[r * stride + blockIdx.x].
__device__ inline void ta_loss_partials(const float4* __restrict__ rec, int64_t P, int runs, double* __restrict__ part,
                                        int64_t stride, int64_t gtid, int64_t gsize, double* lds) {
  for (int r = 0; r < runs; ++r) {
    double v = 0.0;
    for (int64_t n = gtid; n < P; n += gsize) v += (double)rec[r * P + n].w;
    const double t = block_sum(v, lds);
    if (threadIdx.x == 0) part[r * stride + blockIdx.x] = t;
  }
}

// Gradients of one camera for runs r0 .. r0 + G - 1, in every lane of its
// 16-lane row: the records of the camera's pairs, +dL/ds where it is the
// second camera of the pair and -dL/ds where it is the first, summed
// lane-strided over the incidence list and then across the row by a fixed
// butterfly.  Prefix entries past the list's end read pair 0's record and
// add nothing.
template <int G>
__device__ inline void ta_row_grad(const RowList& L, const int32_t* __restrict__ cam_items,
                                   const float4* __restrict__ rec, int64_t P, int r0, int l16, double acc[G][3]) {
  float4 q[G][4];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int j = 0; j < 4; ++j) q[g][j] = rec[(r0 + g) * P + (L.it[j] >= 0 ? (L.it[j] >> 1) : 0)];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    acc[g][0] = acc[g][1] = acc[g][2] = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double sgn = L.it[j] < 0 ? 0.0 : ((L.it[j] & 1) ? 1.0 : -1.0);
      acc[g][0] += sgn * (double)q[g][j].x;
      acc[g][1] += sgn * (double)q[g][j].y;
      acc[g][2] += sgn * (double)q[g][j].z;
    }
  }
  // entries past the first 64 of a long list
  for (int qi = L.lo + 64 + l16; qi < L.hi; qi += 16) {
    const int item = cam_items[qi];
    const double sgn = (item & 1) ? 1.0 : -1.0;
    float4 f[G];
#pragma unroll
    for (int g = 0; g < G; ++g) f[g] = rec[(r0 + g) * P + (item >> 1)];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      acc[g][0] += sgn * (double)f[g].x;
      acc[g][1] += sgn * (double)f[g].y;
      acc[g][2] += sgn * (double)f[g].z;
    }
  }
#pragma unroll
  for (int sh = 8; sh >= 1; sh >>= 1)
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[g][k] += __shfl_xor(acc[g][k], sh);
}

__device__ inline double pick3(const double a[3], int k) { return k == 0 ? a[0] : (k == 1 ? a[1] : a[2]); }

// ------------------------------------------------------------------ target directions

__global__ __launch_bounds__(kBlock) void k_ta_directions(const float* __restrict__ params,
                                                          const int32_t* __restrict__ cams,
                                                          const float* __restrict__ t_rel, int64_t P,
                                                          float* __restrict__ dirs) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= P) return;
  double a1[3], a2[3], t[3], R[3][3];
  load_pose(params, cams[2 * n + 1], a1, a2, t);
  gs_matrix(gs_forward(a1, a2), R);
  double tr[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) tr[k] = (double)t_rel[3 * n + k];
  // -R_j^T t: column k of R dotted with t
#pragma unroll
  for (int k = 0; k < 3; ++k) dirs[3 * n + k] = (float)(-(R[0][k] * tr[0] + R[1][k] * tr[1] + R[2][k] * tr[2]));
}

// ------------------------------------------------------------------ standalone loss + gradient

__global__ __launch_bounds__(kBlock) void k_ta_pair(const float* __restrict__ centres, const int32_t* __restrict__ cams,
                                                    const float* __restrict__ dirs, int64_t P, int32_t N, int runs,
                                                    double invP, float4* __restrict__ rec, double* __restrict__ part,
                                                    int64_t part_stride) {
  __shared__ double lds[kBlock / 64];
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, gsize = (int64_t)gridDim.x * blockDim.x;
  for (int64_t n = gtid; n < P; n += gsize) {
    double d[3];
    load_dir(dirs, n, d);
    ta_pair_runs(centres, N, runs, P, n, cams[2 * n], cams[2 * n + 1], d, invP, rec);
  }
  if (part) ta_loss_partials(rec, P, runs, part, part_stride, gtid, gsize, lds);
}

__global__ __launch_bounds__(kBlock) void k_ta_camera(const int32_t* __restrict__ cam_ptr,
                                                      const int32_t* __restrict__ cam_items,
                                                      const float4* __restrict__ rec, int64_t P, int32_t N, int runs,
                                                      float* __restrict__ grad) {
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = gtid >> 4;
  const int l16 = (int)(gtid & 15);
  if (c >= N) return;   // whole rows leave together: the row exchanges stay within live rows
  const RowList L = row_list(cam_ptr, cam_items, (int)c, l16);
  const int k3 = l16 < 3 ? l16 : 2;
  int r0 = 0;
  for (; r0 + kTaGroup <= runs; r0 += kTaGroup) {
    double acc[kTaGroup][3];
    ta_row_grad<kTaGroup>(L, cam_items, rec, P, r0, l16, acc);
    if (l16 < 3)
#pragma unroll
      for (int g = 0; g < kTaGroup; ++g) grad[((r0 + g) * (int64_t)N + c) * 3 + k3] = (float)pick3(acc[g], k3);
  }
  for (; r0 < runs; ++r0) {
    double acc[1][3];
    ta_row_grad<1>(L, cam_items, rec, P, r0, l16, acc);
    if (l16 < 3) grad[(r0 * (int64_t)N + c) * 3 + k3] = (float)pick3(acc[0], k3);
  }
}

__global__ void k_ta_loss_final(const double* __restrict__ part, int64_t stride, int64_t nblocks, int runs,
                                double invP, double* __restrict__ loss) {
  const int r = threadIdx.x;
  if (r >= runs) return;
  double s = 0.0;
  for (int64_t b = 0; b < nblocks; ++b) s += part[r * stride + b];
  loss[r] = s * invP;
}

// ------------------------------------------------------------------ fused persistent loop

struct TaArgs {
  float* centres;
  float* m;
  float* v;
  const int32_t* cams;
  const float* dirs;
  const int32_t* cam_ptr;
  const int32_t* cam_items;
  float4* rec;
  double* part;
  int64_t part_stride;
  double* trace;
  unsigned* bar;
  int64_t P;
  int32_t N;
  int32_t runs;
  int32_t K;
  double invP, lr, log_frac, b1, b2, eps;
  int64_t lr_step0, lr_total, adam_step0;
};

// Adam steps of one camera (its row) for runs r0 .. r0 + G - 1; lanes 0..2
// own the coordinates.  Parameters and moments are loaded first (they do not
// depend on the records); lanes 3..15 load coordinate 2 and discard it.
template <int G>
__device__ inline void ta_camera_group(const TaArgs& a, const RowList& L, int64_t c, int l16, int r0, double lr,
                                       double bc1, double bc2) {
  const int k3 = l16 < 3 ? l16 : 2;
  float p[G], mq[G], vq[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int64_t idx = ((r0 + g) * (int64_t)a.N + c) * 3 + k3;
    p[g] = a.centres[idx];
    mq[g] = a.m[idx];
    vq[g] = a.v[idx];
  }
  double acc[G][3];
  ta_row_grad<G>(L, a.cam_items, a.rec, a.P, r0, l16, acc);
  if (l16 < 3) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t idx = ((r0 + g) * (int64_t)a.N + c) * 3 + k3;
      a.centres[idx] = adam_update(p[g], (float)pick3(acc[g], k3), mq[g], vq[g], lr, a.b1, a.b2, a.eps, bc1, bc2);
      a.m[idx] = mq[g];
      a.v[idx] = vq[g];
    }
  }
}

__global__ __launch_bounds__(kSolveBlock) void k_ta_solve(TaArgs a) {
  GridBar gb = grid_bar(a.bar);
  __shared__ double lds[kSolveBlock / 64];
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63;
  const int64_t gwave = gtid >> 6, nwaves = gsize >> 6;
  const int row = lane >> 4, l16 = lane & 15;
  // static data of this thread's first pair and this row's first camera,
  // read once instead of once per iteration
  int ci0 = 0, cj0 = 0;
  double d0[3] = {0.0, 0.0, 0.0};
  if (gtid < a.P) {
    ci0 = a.cams[2 * gtid];
    cj0 = a.cams[2 * gtid + 1];
    load_dir(a.dirs, gtid, d0);
  }
  const int64_t c_first = 4 * gwave + row, c_stride = 4 * nwaves;
  RowList L0 = {0, 0, {-1, -1, -1, -1}};
  if (c_first < a.N) L0 = row_list(a.cam_ptr, a.cam_items, (int)c_first, l16);
  StepSched sch(a.log_frac, a.lr_step0, a.lr_total, a.adam_step0, a.b1, a.b2);
  for (int k = 0; k < a.K; ++k) {
    if (gtid < a.P) ta_pair_runs(a.centres, a.N, a.runs, a.P, gtid, ci0, cj0, d0, a.invP, a.rec);
    for (int64_t n = gtid + gsize; n < a.P; n += gsize) {
      double d[3];
      load_dir(a.dirs, n, d);
      ta_pair_runs(a.centres, a.N, a.runs, a.P, n, a.cams[2 * n], a.cams[2 * n + 1], d, a.invP, a.rec);
    }
    if (a.trace) ta_loss_partials(a.rec, a.P, a.runs, a.part, a.part_stride, gtid, gsize, lds);
    grid_barrier(gb);
    if (a.trace && gtid == 0) {
      for (int r = 0; r < a.runs; ++r) {
        double s = 0.0;
        for (int b = 0; b < (int)gridDim.x; ++b) s += a.part[r * a.part_stride + b];
        a.trace[(int64_t)r * a.K + k] = s * a.invP;
      }
    }
    const double lr = a.lr * sch.frac;
    const double bc1 = 1.0 - sch.p1, bc2 = 1.0 - sch.p2;
    sch.next();
    // rows past N skip the camera work as a whole
    for (int64_t c0 = 4 * gwave; c0 < a.N; c0 += c_stride) {
      const int64_t c = c0 + row;
      const bool live = c < a.N;
      const RowList L = c0 == 4 * gwave ? L0 : (live ? row_list(a.cam_ptr, a.cam_items, (int)c, l16)
                                                     : RowList{0, 0, {-1, -1, -1, -1}});
      if (live) {   // whole rows: the row exchanges stay within live rows
        int r0 = 0;
        for (; r0 + kTaGroup <= a.runs; r0 += kTaGroup) ta_camera_group<kTaGroup>(a, L, c, l16, r0, lr, bc1, bc2);
        if (r0 + 2 <= a.runs) {
          ta_camera_group<2>(a, L, c, l16, r0, lr, bc1, bc2);
          r0 += 2;
        }
        if (r0 < a.runs) ta_camera_group<1>(a, L, c, l16, r0, lr, bc1, bc2);
      }
    }
    grid_barrier(gb);
  }
}

// Camera-by-camera variant of the fused loop (the automatic choice): one
// wavefront per camera; each lane evaluates one of the camera's pairs for a
// group of runs and keeps its own side of dL/ds, rounded to float32 as the
// pair records are; the wavefront sums them in a fixed order and lanes
// 0 .. 3G-1 take the Adam steps.  Every pair is evaluated from both of its
// cameras, so no records are exchanged and an iteration needs one grid
// barrier; the centres other wavefronts read are double-buffered by
// iteration parity.
struct TaCamArgs {
  float* centres;    // buffer 0 [runs, N, 3] (the caller's)
  float* alt;        // buffer 1 [runs, N, 3]
  float* m;
  float* v;
  const int32_t* cams;
  const float* dirs;
  const int32_t* cam_ptr;
  const int32_t* cam_items;
  double* part;      // [2, runs, part_stride]
  int64_t part_stride;
  double* trace;
  unsigned* bar;
  int64_t P;
  int32_t N;
  int32_t runs;
  int32_t K;
  double invP, lr, log_frac, b1, b2, eps;
  int64_t lr_step0, lr_total, adam_step0;
};

// Static data of one incidence entry: the entry (pair << 1 | side), both
// cameras and the pair's direction.
struct TaEntry {
  int item, ci, cj;
  float d[3];
};

__device__ inline TaEntry ta_entry(const TaCamArgs& a, int q) {
  TaEntry e;
  e.item = a.cam_items[q];
  const int64_t n = e.item >> 1;
  e.ci = a.cams[2 * n];
  e.cj = a.cams[2 * n + 1];
#pragma unroll
  for (int k = 0; k < 3; ++k) e.d[k] = a.dirs[3 * n + k];
  return e;
}

// One camera for runs r0 .. r0 + G - 1 (G <= 4, so the 3G sums fit the
// 12-value wave reduction).  With `cached`, the lane's first entry of the
// camera is `e0` (read once per launch), so that pass's centre loads depend
// on registers only.  `wl` (the wavefront's loss row in LDS, or NULL)
// gathers the L1 terms of the pairs whose first camera this is, so each
// pair's term is counted once.
template <int G>
__device__ inline void ta_cam_group(const TaCamArgs& a, const float* __restrict__ pr, float* __restrict__ pw,
                                    int64_t c, int lo, int hi, int lane, int r0, double lr, double bc1, double bc2,
                                    double* wl, bool cached, const TaEntry& e0) {
  const int64_t run_stride = (int64_t)a.N * 3;
  // this lane's own coordinate (lanes past 3G repeat the last one)
  const int l3 = lane < 3 * G ? lane : 3 * G - 1;
  const int64_t own = (r0 + l3 / 3) * run_stride + c * 3 + l3 % 3;
  const float p0 = pr[own];
  float mq = a.m[own], vq = a.v[own];
  double acc[12], ls[G];
#pragma unroll
  for (int j = 0; j < 12; ++j) acc[j] = 0.0;
#pragma unroll
  for (int g = 0; g < G; ++g) ls[g] = 0.0;
  for (int q = lo + lane; q < hi; q += 64) {
    TaEntry e;
    if (cached && q == lo + lane)
      e = e0;
    else
      e = ta_entry(a, q);
    const int item = e.item, ci = e.ci, cj = e.cj;
    double d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = (double)e.d[k];
    float oi[G][3], oj[G][3];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        oi[g][k] = pr[(r0 + g) * run_stride + 3 * (int64_t)ci + k];
        oj[g][k] = pr[(r0 + g) * run_stride + 3 * (int64_t)cj + k];
      }
    const double sgn = (item & 1) ? 1.0 : -1.0;
    const double first = (item & 1) ? 0.0 : 1.0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      double sv[3], gr[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) sv[k] = (double)oj[g][k] - (double)oi[g][k];
      const double term = ta_term(sv, d, a.invP, gr);
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[3 * g + k] += sgn * (double)(float)gr[k];
      ls[g] += first * (double)(float)term;
    }
  }
  wave_sum12(acc, lane);
  double gl = acc[0];
#pragma unroll
  for (int j = 1; j < 3 * G; ++j) gl = (l3 == j) ? acc[j] : gl;
  const float pq = adam_update(p0, (float)gl, mq, vq, lr, a.b1, a.b2, a.eps, bc1, bc2);
  if (lane < 3 * G) {
    store_wt(&pw[own], pq);   // read by other workgroups after the barrier
    a.m[own] = mq;
    a.v[own] = vq;
  }
  if (wl) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      double t = ls[g];
#pragma unroll
      for (int sh = 32; sh >= 1; sh >>= 1) t += __shfl_xor(t, sh);
      if (lane == 0) wl[r0 + g] += t;
    }
  }
}

__global__ __launch_bounds__(kSolveBlock) void k_ta_solve_cam(TaCamArgs a) {
  GridBar gb = grid_bar(a.bar);
  __shared__ double wloss[kSolveBlock / 64][kTaMaxRuns];
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t gwave = gtid >> 6, nwaves = gsize >> 6;
  const int64_t RS = (int64_t)a.runs * a.part_stride;
  double* wl = a.trace ? wloss[wv] : nullptr;
  // static data of the first 64 incidence entries of this wavefront's first
  // camera (one per lane), read once for the launch
  TaEntry e0{0, 0, 0, {0.0f, 0.0f, 0.0f}};
  if (gwave < a.N) {
    const int lo = a.cam_ptr[gwave], hi = a.cam_ptr[gwave + 1];
    if (lo + lane < hi) e0 = ta_entry(a, lo + lane);
  }
  StepSched sch(a.log_frac, a.lr_step0, a.lr_total, a.adam_step0, a.b1, a.b2);
  for (int k = 0; k < a.K; ++k) {
    const int rb = k & 1;
    const float* pr = rb ? a.alt : a.centres;
    float* pw = rb ? a.centres : a.alt;
    const double lr = a.lr * sch.frac;
    const double bc1 = 1.0 - sch.p1, bc2 = 1.0 - sch.p2;
    sch.next();
    if (wl) wl[lane] = 0.0;   // kTaMaxRuns == 64: one entry per lane
    // the loop bound is uniform over the wavefront, so the wavefront sums
    // run with every lane present
    for (int64_t c = gwave; c < a.N; c += nwaves) {
      const int lo = a.cam_ptr[c], hi = a.cam_ptr[c + 1];
      int r0 = 0;
      for (; r0 + 4 <= a.runs; r0 += 4) ta_cam_group<4>(a, pr, pw, c, lo, hi, lane, r0, lr, bc1, bc2, wl, c == gwave, e0);
      if (r0 + 2 <= a.runs) {
        ta_cam_group<2>(a, pr, pw, c, lo, hi, lane, r0, lr, bc1, bc2, wl, c == gwave, e0);
        r0 += 2;
      }
      if (r0 < a.runs) ta_cam_group<1>(a, pr, pw, c, lo, hi, lane, r0, lr, bc1, bc2, wl, c == gwave, e0);
    }
    if (a.trace) {
      __syncthreads();
      if ((int)threadIdx.x < a.runs) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += wloss[w][threadIdx.x];
        store_wt(&a.part[rb * RS + threadIdx.x * a.part_stride + blockIdx.x], t);
      }
    }
    // everything other workgroups read after it was written with store_wt
    grid_barrier_wt(gb);
    if (a.trace && gtid == 0) {
      for (int r = 0; r < a.runs; ++r) {
        double t = 0.0;
        for (int b = 0; b < (int)gridDim.x; ++b) t += a.part[rb * RS + r * a.part_stride + b];
        a.trace[(int64_t)r * a.K + k] = t * a.invP;
      }
    }
  }
  // after an odd number of iterations the latest centres are in buffer 1
  if (a.K & 1) {
    const int64_t run_stride = (int64_t)a.N * 3;
    for (int64_t c = gwave; c < a.N; c += nwaves)
      for (int i = lane; i < 3 * a.runs; i += 64) {
        const int64_t idx = (i / 3) * run_stride + c * 3 + i % 3;
        a.centres[idx] = a.alt[idx];
      }
  }
}

// ------------------------------------------------------------------ merge of runs

// Centroid and mean distance to it of each run's centres (one workgroup per
// run, float64, fixed-order sums): stats[r] = (cx, cy, cz, mean norm).
__global__ __launch_bounds__(kBlock) void k_ta_stats(const float* __restrict__ centres, int32_t N,
                                                     double* __restrict__ stats) {
  __shared__ double lds[kBlock / 64];
  __shared__ double cen[3];
  const float* o = centres + (int64_t)blockIdx.x * N * 3;
  double s[3] = {0.0, 0.0, 0.0};
  for (int c = threadIdx.x; c < N; c += blockDim.x)
#pragma unroll
    for (int k = 0; k < 3; ++k) s[k] += (double)o[3 * c + k];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double t = block_sum(s[k], lds);
    if (threadIdx.x == 0) cen[k] = t / (double)N;
  }
  __syncthreads();
  double sn = 0.0;
  for (int c = threadIdx.x; c < N; c += blockDim.x) {
    const double dx = (double)o[3 * c] - cen[0], dy = (double)o[3 * c + 1] - cen[1], dz = (double)o[3 * c + 2] - cen[2];
    sn += sqrt(dx * dx + dy * dy + dz * dz);
  }
  const double t = block_sum(sn, lds);
  if (threadIdx.x == 0) {
    double* st = stats + 4 * (int64_t)blockIdx.x;
    st[0] = cen[0];
    st[1] = cen[1];
    st[2] = cen[2];
    st[3] = t / (double)N;
  }
}

// Per camera (one 16-lane row): the mean L1 term of its pairs in every run,
// the run with the lowest mean (the first among equals), and that run's
// centre moved to its run's centroid and scaled to unit mean norm.
__global__ __launch_bounds__(kBlock) void k_ta_merge(const float* __restrict__ centres, const int32_t* __restrict__ cams,
                                                     const float* __restrict__ dirs, const int32_t* __restrict__ cam_ptr,
                                                     const int32_t* __restrict__ cam_items,
                                                     const double* __restrict__ stats, int32_t N, int runs,
                                                     double* __restrict__ cam_loss, int32_t* __restrict__ choice,
                                                     float* __restrict__ merged) {
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = gtid >> 4;
  const int l16 = (int)(gtid & 15);
  if (c >= N) return;   // whole rows leave together
  const int lo = cam_ptr[c], hi = cam_ptr[c + 1];
  const double cnt = (double)(hi - lo);
  int best = 0;
  double best_v = 0.0;
  for (int r = 0; r < runs; ++r) {
    const float* o = centres + (int64_t)r * N * 3;
    double acc = 0.0;
    for (int q = lo + l16; q < hi; q += 16) {
      const int64_t n = cam_items[q] >> 1;
      double d[3];
      load_dir(dirs, n, d);
      acc += ta_term_at(o + 3 * (int64_t)cams[2 * n], o + 3 * (int64_t)cams[2 * n + 1], d);
    }
#pragma unroll
    for (int s = 8; s >= 1; s >>= 1) acc += __shfl_xor(acc, s);
    const double mean = hi > lo ? acc / cnt : 0.0;
    if (cam_loss && l16 == 0) cam_loss[(int64_t)r * N + c] = mean;
    if (r == 0 || mean < best_v) {
      best = r;
      best_v = mean;
    }
  }
  if (l16 < 3) {
    const double* st = stats + 4 * best;
    const double x = (double)centres[((int64_t)best * N + c) * 3 + l16] - st[l16];
    merged[c * 3 + l16] = (float)(st[3] > 0.0 ? x / st[3] : x);
  }
  if (choice && l16 == 0) choice[c] = best;
}

// ------------------------------------------------------------------ poses from centres

// (a1, a2, t = -R o) per camera: the epipolar parameters of rotations given
// as 6D parameters and camera centres o (R by Gram-Schmidt, float64).
__global__ __launch_bounds__(kBlock) void k_poses_from_centres(const float* __restrict__ p6,
                                                               const float* __restrict__ centres, int32_t N,
                                                               float* __restrict__ p9) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  double a1[3], a2[3], R[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    a1[k] = (double)p6[6 * c + k];
    a2[k] = (double)p6[6 * c + 3 + k];
  }
  gs_matrix(gs_forward(a1, a2), R);
  const double o[3] = {(double)centres[3 * c], (double)centres[3 * c + 1], (double)centres[3 * c + 2]};
#pragma unroll
  for (int k = 0; k < 6; ++k) p9[9 * c + k] = p6[6 * c + k];
#pragma unroll
  for (int a = 0; a < 3; ++a) p9[9 * c + 6 + a] = (float)(-(R[a][0] * o[0] + R[a][1] * o[1] + R[a][2] * o[2]));
}

// ------------------------------------------------------------------ host side

fm_status ta_check(fm_ctx* ctx, fm_scene* s, const char* fn) {
  if (!s) return fm_fail(ctx, FM_EINVAL, "%s: scene is NULL", fn);
  if (s->ctx != ctx) return fm_fail(ctx, FM_EINVAL, "%s: scene belongs to another context", fn);
  return FM_OK;
}

fm_status ta_check_runs(fm_ctx* ctx, const char* fn, int32_t runs) {
  if (runs < 1 || runs > kTaMaxRuns) return fm_fail(ctx, FM_EINVAL, "%s: runs must be in [1, %d]", fn, kTaMaxRuns);
  return FM_OK;
}

// Workspace for `runs` runs (records, loss partials, run statistics), grown
// on demand: a larger request synchronises the device and reallocates.
fm_status ta_reserve(fm_ctx* ctx, fm_scene* s, int runs) {
  if (s->ta_coop_blocks <= 0) {
    int per_cu = 0;
    FM_HIP_TRY(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ta_solve, kSolveBlock, 0));
    int per_cu_cam = 0;
    FM_HIP_TRY(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_cam, k_ta_solve_cam, kSolveBlock, 0));
    if (per_cu_cam < per_cu) per_cu = per_cu_cam;
    s->ta_coop_blocks = per_cu * ctx->num_cu;
    if (s->ta_coop_blocks <= 0) return fm_fail(ctx, FM_ECOOP, "cannot size the cooperative translation kernel");
  }
  if (runs <= s->ta_runs_cap) return FM_OK;
  int64_t part = (int64_t)grid_for(s->P, kBlock);
  if (part < s->ta_coop_blocks) part = s->ta_coop_blocks;
  FM_HIP_TRY(ctx, hipDeviceSynchronize());
  (void)hipFree(s->ta_rec);
  (void)hipFree(s->ta_part);
  (void)hipFree(s->ta_stats);
  (void)hipFree(s->ta_alt);
  s->ta_rec = nullptr;
  s->ta_part = nullptr;
  s->ta_stats = nullptr;
  s->ta_alt = nullptr;
  s->ta_runs_cap = 0;
  const int64_t P1 = s->P > 0 ? s->P : 1;
  const int64_t N1 = s->N > 0 ? s->N : 1;
  // loss partials: two sets (the camera loop alternates them by iteration)
  if (hipMalloc(&s->ta_rec, sizeof(float4) * runs * P1) != hipSuccess ||
      hipMalloc(&s->ta_part, sizeof(double) * 2 * runs * part) != hipSuccess ||
      hipMalloc(&s->ta_stats, sizeof(double) * 4 * runs) != hipSuccess ||
      hipMalloc(&s->ta_alt, sizeof(float) * 3 * runs * N1) != hipSuccess) {
    (void)hipGetLastError();
    return fm_fail(ctx, FM_ENOMEM, "translation workspace for %d runs: allocation failed", runs);
  }
  s->ta_part_cap = part;
  s->ta_runs_cap = runs;
  return FM_OK;
}

}  // namespace

extern "C" fm_status fm_translation_directions(fm_ctx* ctx, fm_scene* s, const float* params, const float* t_rel,
                                               float* dirs, fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  fm_status rc = ta_check(ctx, s, "fm_translation_directions");
  if (rc != FM_OK) return rc;
  if (s->P == 0) return FM_OK;
  if (!params || !t_rel || !dirs) return fm_fail(ctx, FM_EINVAL, "fm_translation_directions: NULL argument");
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipLaunchKernelGGL(k_ta_directions, dim3(grid_for(s->P, kBlock)), dim3(kBlock), 0, (hipStream_t)stream, params,
                     s->pair_cams, t_rel, s->P, dirs);
  FM_CHECK_LAUNCH(ctx);
  return FM_OK;
}

extern "C" fm_status fm_translation_loss_grad(fm_ctx* ctx, fm_scene* s, const float* dirs, int32_t runs,
                                              const float* centres, double* loss, float* grad, fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  fm_status rc = ta_check(ctx, s, "fm_translation_loss_grad");
  if (rc != FM_OK) return rc;
  if ((rc = ta_check_runs(ctx, "fm_translation_loss_grad", runs)) != FM_OK) return rc;
  if ((s->P > 0 && !dirs) || (s->N > 0 && !centres))
    return fm_fail(ctx, FM_EINVAL, "fm_translation_loss_grad: NULL argument");
  if (!loss && !grad) return FM_OK;
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  if (s->P == 0) {
    if (loss) FM_HIP_TRY(ctx, hipMemsetAsync(loss, 0, sizeof(double) * runs, st));
    if (grad && s->N > 0) FM_HIP_TRY(ctx, hipMemsetAsync(grad, 0, sizeof(float) * 3 * runs * (size_t)s->N, st));
    return FM_OK;
  }
  if ((rc = ta_reserve(ctx, s, runs)) != FM_OK) return rc;
  const double invP = 1.0 / (double)s->P;
  const unsigned gp = grid_for(s->P, kBlock);
  {
    fm_timed timer(ctx, FM_K_TA_PAIR, st);
    hipLaunchKernelGGL(k_ta_pair, dim3(gp), dim3(kBlock), 0, st, centres, s->pair_cams, dirs, s->P, s->N, (int)runs,
                       invP, reinterpret_cast<float4*>(s->ta_rec), loss ? s->ta_part : nullptr, s->ta_part_cap);
    FM_CHECK_LAUNCH(ctx);
  }
  if (loss) {
    hipLaunchKernelGGL(k_ta_loss_final, dim3(1), dim3(64), 0, st, s->ta_part, s->ta_part_cap, (int64_t)gp, (int)runs,
                       invP, loss);
    FM_CHECK_LAUNCH(ctx);
  }
  if (grad && s->N > 0) {
    fm_timed timer(ctx, FM_K_TA_CAMERA, st);
    hipLaunchKernelGGL(k_ta_camera, dim3(grid_for((int64_t)s->N * 16, kBlock)), dim3(kBlock), 0, st, s->cam_ptr,
                       s->cam_items, reinterpret_cast<const float4*>(s->ta_rec), s->P, s->N, (int)runs, grad);
    FM_CHECK_LAUNCH(ctx);
  }
  return FM_OK;
}

extern "C" fm_status fm_translation_solve(fm_ctx* ctx, fm_scene* s, const float* dirs, int32_t runs, float* centres,
                                          float* m, float* v, int32_t K, const fm_adam_cfg* cfg, double* loss_trace,
                                          fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  fm_status rc = ta_check(ctx, s, "fm_translation_solve");
  if (rc != FM_OK) return rc;
  if ((rc = ta_check_runs(ctx, "fm_translation_solve", runs)) != FM_OK) return rc;
  if (!cfg || (s->P > 0 && !dirs) || (s->N > 0 && (!centres || !m || !v)))
    return fm_fail(ctx, FM_EINVAL, "fm_translation_solve: NULL argument");
  if (K < 0) return fm_fail(ctx, FM_EINVAL, "fm_translation_solve: K < 0");
  if (cfg->lr_total_steps <= 0 || cfg->lr_step0 < 0 || cfg->adam_step0 < 0 || !(cfg->lr_final_frac > 0.0f) ||
      !(cfg->lr_t >= 0.0f) ||
      !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f && cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f && cfg->eps >= 0.0f))
    return fm_fail(ctx, FM_EINVAL, "fm_translation_solve: bad Adam configuration");
  if (K == 0 || s->N == 0) return FM_OK;
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  if ((rc = ta_reserve(ctx, s, runs)) != FM_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  // sized like the epipolar loop: about one pair per thread or one 16-lane
  // row per camera, capped at 16 workgroups while runs x P < 32k and at 192
  // above, and at the co-resident limit
  int64_t want = grid_for(s->P, kSolveBlock);
  const int64_t want_c = grid_for((int64_t)s->N * 16, kSolveBlock);
  if (want_c > want) want = want_c;
  const int64_t cap = (int64_t)runs * s->P < 32768 ? 16 : 192;
  if (want > cap) want = cap;
  if (cfg->blocks > 0) want = cfg->blocks;
  if (want < 1) want = 1;
  if (want > s->ta_coop_blocks) want = s->ta_coop_blocks;
  if (want > s->ta_part_cap) want = s->ta_part_cap;
  TaArgs a;
  a.centres = centres; a.m = m; a.v = v;
  a.cams = s->pair_cams; a.dirs = dirs; a.cam_ptr = s->cam_ptr; a.cam_items = s->cam_items;
  a.rec = reinterpret_cast<float4*>(s->ta_rec); a.part = s->ta_part; a.part_stride = s->ta_part_cap;
  a.trace = loss_trace; a.bar = s->bar;
  a.P = s->P; a.N = s->N; a.runs = runs; a.K = K;
  a.invP = s->P > 0 ? 1.0 / (double)s->P : 0.0;
  a.lr = cfg->lr_t; a.log_frac = log((double)cfg->lr_final_frac);
  a.b1 = cfg->beta1; a.b2 = cfg->beta2; a.eps = cfg->eps;
  a.lr_step0 = cfg->lr_step0; a.lr_total = cfg->lr_total_steps; a.adam_step0 = cfg->adam_step0;
  void* args[] = {&a};
  FM_HIP_TRY(ctx, fm_bar_reset(s->bar, st));
  if (cfg->blocks <= 0) {
    // automatic grid: the camera loop, one wavefront per camera up to the
    // co-resident limit (cameras strided beyond it).  Unlike the epipolar
    // pair term, this one is cheap enough to evaluate twice at any size
    // measured: on the 5,000-camera street graph (185k pairs) 24.0 against
    // 27.3 us per iteration for 4 runs
    const CamGrid cg = cam_grid(s->N, s->ta_coop_blocks, ctx->num_cu);
    int64_t want_cam = cg.blocks;
    if (want_cam > s->ta_part_cap) want_cam = s->ta_part_cap;
    TaCamArgs ca;
    ca.centres = centres; ca.alt = s->ta_alt; ca.m = m; ca.v = v;
    ca.cams = s->pair_cams; ca.dirs = dirs; ca.cam_ptr = s->cam_ptr; ca.cam_items = s->cam_items;
    ca.part = s->ta_part; ca.part_stride = s->ta_part_cap; ca.trace = loss_trace; ca.bar = s->bar;
    ca.P = s->P; ca.N = s->N; ca.runs = runs; ca.K = K;
    ca.invP = a.invP; ca.lr = a.lr; ca.log_frac = a.log_frac; ca.b1 = a.b1; ca.b2 = a.b2; ca.eps = a.eps;
    ca.lr_step0 = a.lr_step0; ca.lr_total = a.lr_total; ca.adam_step0 = a.adam_step0;
    void* cargs[] = {&ca};
    fm_timed timer(ctx, FM_K_TA_SOLVE, st);
    hipError_t e = hipLaunchCooperativeKernel((const void*)k_ta_solve_cam, dim3((unsigned)want_cam),
                                              dim3(cg.threads), cargs, 0, st);
    if (e != hipSuccess) return fm_fail(ctx, FM_ECOOP, "cooperative launch failed: %s", hipGetErrorString(e));
    return FM_OK;
  }
  fm_timed timer(ctx, FM_K_TA_SOLVE, st);
  hipError_t e = hipLaunchCooperativeKernel((const void*)k_ta_solve, dim3((unsigned)want), dim3(kSolveBlock), args, 0, st);
  if (e != hipSuccess) return fm_fail(ctx, FM_ECOOP, "cooperative launch failed: %s", hipGetErrorString(e));
  return FM_OK;
}

extern "C" fm_status fm_translation_merge(fm_ctx* ctx, fm_scene* s, const float* dirs, int32_t runs,
                                          const float* centres, float* merged, int32_t* choice, double* cam_loss,
                                          fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  fm_status rc = ta_check(ctx, s, "fm_translation_merge");
  if (rc != FM_OK) return rc;
  if ((rc = ta_check_runs(ctx, "fm_translation_merge", runs)) != FM_OK) return rc;
  if ((s->P > 0 && !dirs) || (s->N > 0 && (!centres || !merged)))
    return fm_fail(ctx, FM_EINVAL, "fm_translation_merge: NULL argument");
  if (s->N == 0) return FM_OK;
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  if ((rc = ta_reserve(ctx, s, runs)) != FM_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_ta_stats, dim3(runs), dim3(kBlock), 0, st, centres, s->N, s->ta_stats);
  FM_CHECK_LAUNCH(ctx);
  hipLaunchKernelGGL(k_ta_merge, dim3(grid_for((int64_t)s->N * 16, kBlock)), dim3(kBlock), 0, st, centres,
                     s->pair_cams, dirs, s->cam_ptr, s->cam_items, s->ta_stats, s->N, (int)runs, cam_loss, choice,
                     merged);
  FM_CHECK_LAUNCH(ctx);
  return FM_OK;
}

extern "C" fm_status fm_poses_from_centres(fm_ctx* ctx, int32_t N, const float* params6, const float* centres,
                                           float* params9, fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  if (N < 0) return fm_fail(ctx, FM_ESHAPE, "fm_poses_from_centres: N < 0");
  if (N == 0) return FM_OK;
  if (!params6 || !centres || !params9) return fm_fail(ctx, FM_EINVAL, "fm_poses_from_centres: NULL argument");
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipLaunchKernelGGL(k_poses_from_centres, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, (hipStream_t)stream, params6,
                     centres, N, params9);
  FM_CHECK_LAUNCH(ctx);
  return FM_OK;
}
