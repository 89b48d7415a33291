// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_ext.h>

#include "fastmap_hip.h"

// Matches per feature work item: one wavefront of 64 lanes, 16 matches per lane.
constexpr int kLanes = 64;
constexpr int kPerLane = 16;
constexpr int kChunk = kLanes * kPerLane;
// Rows per lane of a Gram work item, for a wavefront on one chunk of a large
// pair (64 lanes) and for a wavefront on four small pairs (16 lanes each):
// 64 for BF16 coordinates (the pass is bound by vector ALU issue there, and
// longer items spread each wavefront's 36-value reduction over more
// matches), 16 otherwise (the FP32 pass waits on memory, and more, shorter
// wavefronts hide that better).
constexpr int big_rows(int dt) { return dt == FM_BF16 ? 4 * kPerLane : kPerLane; }
constexpr int group_rows(int dt) { return dt == FM_BF16 ? 4 * kPerLane : kPerLane; }
// Pairs with at most small_max(dt) matches share a wavefront, four at a time.
constexpr int small_max(int dt) { return 16 * group_rows(dt); }
// Wavefronts per block of the Gram kernels.
constexpr int kGramWaves = 4;
// Threads per block of the per-pair and per-camera kernels.
constexpr int kBlock = 256;
// Threads per workgroup of the persistent solve (eight wavefronts: fewer,
// larger workgroups make its grid barriers cheaper).
constexpr int kSolveBlock = 512;
// Threads per workgroup of the camera loops (the epipolar one always, the
// translation, rotation and focal ones while a workgroup per CU suffices):
// four wavefronts, so that the loops' wavefronts (one per camera) spread
// over twice as many CUs as with eight.  Medium helix scene, µs per
// iteration of the epipolar loop: 512 threads 8.2, 256 7.1, 128 7.6 (more
// workgroups make each grid barrier dearer); translation (4 runs) 5.20 ->
// 4.63, rotation 6.08 -> 5.05, focal 9.39 -> 7.34 going from 512 to 256.
constexpr int kCamBlock = 256;

// Workgroup size and count of a camera-by-camera loop compiled for up to
// kSolveBlock threads (one wavefront per camera): kCamBlock-thread
// workgroups while they fit one to a CU (the wavefronts then spread over
// twice as many CUs: one per SIMD instead of two), else kSolveBlock-thread
// workgroups up to `coop` co-resident (cameras strided beyond them).
struct CamGrid {
  int threads;
  int64_t blocks;
};
inline CamGrid cam_grid(int64_t N, int64_t coop, int num_cu) {
  const int64_t small = (N * 64 + kCamBlock - 1) / kCamBlock;
  if (small <= num_cu) return CamGrid{kCamBlock, small > 0 ? small : 1};
  int64_t b = (N * 64 + kSolveBlock - 1) / kSolveBlock;
  if (b > coop) b = coop;
  return CamGrid{kSolveBlock, b};
}
// Integer counters the IRLS pass spreads its kept-match counts over (one
// 128-byte line each, so concurrent atomics rarely meet on one address).
constexpr int kKeptSlots = 256;

// Kernel identifiers of the optional launch timing (fm_profile_*).
enum { FM_K_GRAM = 0, FM_K_SOLVE = 1, FM_K_ESSENTIALS = 2, FM_K_FINALIZE = 3, FM_K_PAIR = 4, FM_K_CAMERA = 5,
       FM_K_TA_SOLVE = 6, FM_K_TA_PAIR = 7, FM_K_TA_CAMERA = 8, FM_K_RA_SOLVE = 9, FM_K_RA_PAIR = 10,
       FM_K_RA_CAMERA = 11, FM_K_RA_INIT = 12, FM_K_TS_SEARCH = 13, FM_K_FO_PAIR = 14, FM_K_FO_CAMERA = 15,
       FM_K_FO_SOLVE = 16, FM_K_GRAM_CALL = 17,
       FM_K_COUNT = 18 };

struct fm_timing {
  int kernel;
  hipEvent_t start, stop;
};

struct fm_ctx {
  int device = 0;
  int num_cu = 0;
  std::string err;
  bool profile = false;
  std::vector<fm_timing> timings;    // recorded launches (profiling on)
  std::vector<hipEvent_t> event_pool;
  void* ws = nullptr;                // grow-only workspace (MLP gradient slots)
  size_t ws_bytes = 0;
  bool check = false;                // opt-in device-side data checks (fm_set_check)
  unsigned* check_flag = nullptr;    // [1] device: FM_CHECK_* bits raised since the last fm_check
};

// Timing of one kernel launch when profiling is on.  By default the two
// events bracket the launch on its stream; with `at_dispatch` the caller
// hands a and b to hipExtLaunchKernelGGL, which records them at the start
// and end of the kernel itself (no dispatch latency in the interval).
struct fm_timed {
  fm_ctx* ctx;
  int kernel;
  hipStream_t st;
  bool at_dispatch;
  hipEvent_t a = nullptr, b = nullptr;
  fm_timed(fm_ctx* c, int k, hipStream_t s, bool dispatch = false);
  ~fm_timed();
};

struct fm_scene {
  fm_ctx* ctx = nullptr;
  int64_t P = 0, M = 0;
  int32_t N = 0;
  const int64_t* offsets = nullptr;
  const int32_t* pair_cams = nullptr;
  const void* uv = nullptr;
  fm_dtype dtype = FM_F32;
  // derived index data
  int64_t n_wi = 0;               // Gram work items
  int64_t* wi_off = nullptr;      // [P+1] first work item of each pair
  int32_t* wi_pair = nullptr;     // [n_wi] pair of each work item
  // Gram pass plan (built at set-up)
  int64_t n_big = 0;              // chunk work items of pairs with more than small_max(dtype) matches
  int32_t* big_pair = nullptr;    // [n_big] pair of each chunk
  int32_t* big_chunk = nullptr;   // [n_big] chunk index within its pair
  int32_t* big_slot = nullptr;    // [n_big] partial slot of the chunk (-1: the chunk is its whole pair)
  int64_t chunk = kChunk;         // matches per big work item (kLanes * big_rows(dtype))
  int64_t n_partials = 0;         // chunk partials of pairs spanning several chunks
  int64_t n_groups = 0;           // wavefronts of four pairs with 0..small_max(dtype) matches
  int32_t* groups = nullptr;      // [4 n_groups] pair ids (-1: none)
  int64_t n_multi = 0;            // pairs spanning more than one chunk
  int64_t n_empty = 0;            // pairs without matches (in groups, zero rows)
  int32_t* multi = nullptr;       // [n_multi] pairs spanning several chunks
  int64_t* multi_first = nullptr; // [n_multi] first partial slot of each multi pair
  unsigned long long* kept_slots = nullptr;  // [kKeptSlots * 16] kept-match counters, one per 128-B line
  int32_t* cam_ptr = nullptr;     // [N+1] incidence list offsets
  int32_t* cam_items = nullptr;   // [2P] 2*pair + side (0: camera is i_n, 1: j_n), pair order
  int32_t* pair_slot = nullptr;   // [2P] position of item 2*pair + side in cam_items
  // workspace
  float* partials = nullptr;      // [n_big, 36]
  double* ess = nullptr;          // [P, 9] essential matrices (reweight)
  float* contrib = nullptr;       // [P, 24] per-pair gradient records
  float* fo_rec = nullptr;        // [P, 2] per-pair focal-scale gradient records (side i, side j)
  double* loss_part = nullptr;    // [loss_part_cap]
  double* rot = nullptr;          // [2, N, 9] rotations of the current poses (fused solve; two buffers)
  float* params_alt = nullptr;    // [N, 10] second parameter buffer of the camera loops ([N, 9] poses, then [N] focal scales)
  int64_t loss_part_cap = 0;
  unsigned* bar = nullptr;        // [kBarWords] grid barriers of the persistent loops (layout at kBarWords)
  int coop_blocks = 0;            // max co-resident workgroups of the fused pair loop (kSolveBlock threads)
  int coop_blocks_cam = 0;        // max co-resident workgroups of the fused camera loop (kCamBlock threads)
  // translation averaging workspace, grown on demand by the translation calls
  int32_t ta_runs_cap = 0;        // runs the workspace holds
  int64_t ta_part_cap = 0;        // loss partials per run
  void* ta_rec = nullptr;         // [ta_runs_cap, P] float4 per-pair records: dL/ds and the pair's L1 term
  double* ta_part = nullptr;      // [2, ta_runs_cap, ta_part_cap] per-workgroup loss partials
  float* ta_alt = nullptr;        // [ta_runs_cap, N, 3] second centre buffer of the camera loop
  double* ta_stats = nullptr;     // [ta_runs_cap, 4] centroid and mean norm of each run
  int ta_coop_blocks = 0;         // max co-resident blocks of the translation loop
  int fo_coop_blocks = 0;         // max co-resident blocks of the focal loop
  int ra_coop_blocks = 0;         // max co-resident blocks of the rotation loop
  // rotation initialisation workspace (Lanczos basis), grown on demand
  int64_t lz_cap = 0;             // doubles held by lz
  double* lz = nullptr;           // basis [m+1, 3N], work vector, dots, tridiagonal, Ritz coefficients
  int lz_coop_blocks = 0;         // max co-resident blocks of the Lanczos kernel
};

// Check mode: scans n float32 (f64 = false) or float64 values at p for a
// non-finite one and raises `bit` in ctx->check_flag (no-op when check mode
// is off).
fm_status fm_check_finite(fm_ctx* ctx, hipStream_t st, const void* p, int64_t n, bool f64, unsigned bit);
// E_n of every pair at `params` into the scene's workspace (gram.hip); in
// check mode it also flags degenerate pairs and non-finite parameters.
fm_status fm_launch_essentials(fm_scene* s, const float* params, hipStream_t st);

// Error reporting helpers: set ctx->err and return the status.
fm_status fm_fail(fm_ctx* ctx, fm_status st, const char* fmt, ...);

#define FM_HIP_TRY(ctx, expr)                                                        \
  do {                                                                               \
    hipError_t _e = (expr);                                                          \
    if (_e != hipSuccess)                                                            \
      return fm_fail((ctx), FM_EHIP, "%s failed: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

#define FM_CHECK_LAUNCH(ctx)                                                         \
  do {                                                                               \
    hipError_t _e = hipGetLastError();                                               \
    if (_e != hipSuccess)                                                            \
      return fm_fail((ctx), FM_EHIP, "kernel launch failed: %s", hipGetErrorString(_e)); \
  } while (0)

static inline unsigned grid_for(int64_t n, int block) {
  return (unsigned)((n + block - 1) / block);
}

// ------------------------------------------------------------------ device helpers

// Gram-Schmidt of the 6D rotation parameters (a1, a2) into the columns
// b1, b2, b3 of R, in float64.  Also returns |a1|, |u2|, their reciprocals
// and b1.a2 for the adjoint.
struct Gs {
  double b1[3], b2[3], b3[3];
  double n1, n2, r1, r2, d12;
};

__device__ inline Gs gs_forward(const double a1[3], const double a2[3]) {
  Gs g;
  g.n1 = sqrt(a1[0] * a1[0] + a1[1] * a1[1] + a1[2] * a1[2]);
  g.r1 = 1.0 / g.n1;
  for (int k = 0; k < 3; ++k) g.b1[k] = a1[k] * g.r1;
  g.d12 = g.b1[0] * a2[0] + g.b1[1] * a2[1] + g.b1[2] * a2[2];
  double u2[3];
  for (int k = 0; k < 3; ++k) u2[k] = a2[k] - g.d12 * g.b1[k];
  g.n2 = sqrt(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
  g.r2 = 1.0 / g.n2;
  for (int k = 0; k < 3; ++k) g.b2[k] = u2[k] * g.r2;
  g.b3[0] = g.b1[1] * g.b2[2] - g.b1[2] * g.b2[1];
  g.b3[1] = g.b1[2] * g.b2[0] - g.b1[0] * g.b2[2];
  g.b3[2] = g.b1[0] * g.b2[1] - g.b1[1] * g.b2[0];
  return g;
}

// R[r][c] = b_c[r]
__device__ inline void gs_matrix(const Gs& g, double R[3][3]) {
  for (int r = 0; r < 3; ++r) {
    R[r][0] = g.b1[r];
    R[r][1] = g.b2[r];
    R[r][2] = g.b3[r];
  }
}

__device__ inline void load_pose(const float* params, int c, double a1[3], double a2[3], double t[3]) {
  const int64_t b = (int64_t)c * 9;
  for (int k = 0; k < 3; ++k) {
    a1[k] = (double)params[b + k];
    a2[k] = (double)params[b + 3 + k];
    t[k] = (double)params[b + 6 + k];
  }
}

// Relative pose and essential matrix of pair (i, j) in float64:
// R_ij = R_j R_i^T, s = t_j - R_ij t_i, th = s/|s|, E = [th]_x R_ij.
// Returns |s| (0 for a degenerate pair, in which case E = 0).
__device__ inline double pair_essential(const double Ri[3][3], const double ti[3],
                                        const double Rj[3][3], const double tj[3],
                                        double Rij[3][3], double th[3], double E[3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      Rij[a][b] = Rj[a][0] * Ri[b][0] + Rj[a][1] * Ri[b][1] + Rj[a][2] * Ri[b][2];
  double s[3];
  for (int a = 0; a < 3; ++a)
    s[a] = tj[a] - (Rij[a][0] * ti[0] + Rij[a][1] * ti[1] + Rij[a][2] * ti[2]);
  double ns = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
  double inv = ns > 0.0 ? 1.0 / ns : 0.0;
  for (int a = 0; a < 3; ++a) th[a] = s[a] * inv;
  // rows of [th]_x
  const double T[3][3] = {{0.0, -th[2], th[1]}, {th[2], 0.0, -th[0]}, {-th[1], th[0], 0.0}};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      E[a][b] = T[a][0] * Rij[0][b] + T[a][1] * Rij[1][b] + T[a][2] * Rij[2][b];
  return ns;
}

// Adjoint of E = [th]_x R_ij (th = s/|s|, s = t_j - R_ij t_i, R_ij = R_j R_i^T)
// from G = dL/dE to the pair's record [dL/dR_i (3x3 row-major), dL/dt_i,
// dL/dR_j, dL/dt_j] (float32); ns = |s| > 0.
__device__ inline void essential_adjoint(const double G[3][3], const double th[3], double ns, const double Rij[3][3],
                                         const double Ri[3][3], const double Rj[3][3], const double ti[3],
                                         float* __restrict__ rec) {
  const double T[3][3] = {{0.0, -th[2], th[1]}, {th[2], 0.0, -th[0]}, {-th[1], th[0], 0.0}};
  double A[3][3], dRij[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      A[a][b] = G[a][0] * Rij[b][0] + G[a][1] * Rij[b][1] + G[a][2] * Rij[b][2];
      dRij[a][b] = T[0][a] * G[0][b] + T[1][a] * G[1][b] + T[2][a] * G[2][b];
    }
  // through T = [th]_x, th = s/|s|, s = t_j - R_ij t_i
  double gth[3] = {A[2][1] - A[1][2], A[0][2] - A[2][0], A[1][0] - A[0][1]};
  const double dp = th[0] * gth[0] + th[1] * gth[1] + th[2] * gth[2];
  const double rns = 1.0 / ns;
  double gs[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) gs[k] = (gth[k] - dp * th[k]) * rns;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) dRij[a][b] -= gs[a] * ti[b];
  // R_ij = R_j R_i^T: dR_j = dRij R_i, dR_i = dRij^T R_j
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      rec[12 + 3 * a + b] = (float)(dRij[a][0] * Ri[0][b] + dRij[a][1] * Ri[1][b] + dRij[a][2] * Ri[2][b]);
      rec[3 * a + b] = (float)(dRij[0][a] * Rj[0][b] + dRij[1][a] * Rj[1][b] + dRij[2][a] * Rj[2][b]);
    }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    rec[21 + a] = (float)gs[a];
    rec[9 + a] = (float)(-(Rij[0][a] * gs[0] + Rij[1][a] * gs[1] + Rij[2][a] * gs[2]));
  }
}

// The adjoint of E = [th]_x R_ij in the form the fused loops' camera updates
// use.  The loss depends on R_i, R_j only through R_ij = R_j R_i^T, so the
// body-frame rotation gradients of the two cameras are opposite: om =
// vee(skew(R_j^T dL/dR_j)) for camera j and -om for camera i.  With
// R_j^T dL/dR_j = R_j^T dRij R_i (dRij = dL/dR_ij) and R_j = R_ij R_i,
// om = R_i^T vee(skew(R_ij^T dRij)) (vee(skew(Q^T A Q)) = Q^T vee(skew(A))
// for a rotation Q), so R_j is not needed here.  Only that tangent part of
// dL/dR reaches the 6D parameters (every change of the parameters moves R
// along SO(3)), so a camera's update rebuilds dL/dR from the sum of its
// pairs' om (omega_grad).  Also dL/dt_i and dL/dt_j.  ns = |s| > 0.
__device__ inline void essential_adjoint_omega(const double G[3][3], const double th[3], double ns,
                                               const double Rij[3][3], const double Ri[3][3], const double ti[3],
                                               double om[3], double dti[3], double dtj[3]) {
  const double T[3][3] = {{0.0, -th[2], th[1]}, {th[2], 0.0, -th[0]}, {-th[1], th[0], 0.0}};
  double A[3][3], dRij[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      A[a][b] = G[a][0] * Rij[b][0] + G[a][1] * Rij[b][1] + G[a][2] * Rij[b][2];
      dRij[a][b] = T[0][a] * G[0][b] + T[1][a] * G[1][b] + T[2][a] * G[2][b];
    }
  const double gth[3] = {A[2][1] - A[1][2], A[0][2] - A[2][0], A[1][0] - A[0][1]};
  const double dp = th[0] * gth[0] + th[1] * gth[1] + th[2] * gth[2];
  const double rns = 1.0 / ns;
  double gs[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) gs[k] = (gth[k] - dp * th[k]) * rns;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) dRij[a][b] -= gs[a] * ti[b];
  // w = vee(skew(R_ij^T dRij)) from the off-diagonal entries of R_ij^T dRij
  auto K = [&](int a, int b) { return Rij[0][a] * dRij[0][b] + Rij[1][a] * dRij[1][b] + Rij[2][a] * dRij[2][b]; };
  const double w[3] = {0.5 * (K(2, 1) - K(1, 2)), 0.5 * (K(0, 2) - K(2, 0)), 0.5 * (K(1, 0) - K(0, 1))};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    om[a] = Ri[0][a] * w[0] + Ri[1][a] * w[1] + Ri[2][a] * w[2];
    dtj[a] = gs[a];
    dti[a] = -(Rij[0][a] * gs[0] + Rij[1][a] * gs[1] + Rij[2][a] * gs[2]);
  }
}

// Symmetric monomial index q(a, c) of x~[a] x~[c] in p = (u^2, uv, v^2, u, v, 1).
__device__ __host__ constexpr int mono_q(int a, int c) {
  return (a == c) ? (a == 0 ? 0 : (a == 1 ? 2 : 5))
                  : ((a + c) == 1 ? 1 : ((a + c) == 2 ? 3 : 4));
}

// Incidence list of one camera as one 16-lane row reads it: the list bounds
// and this lane's first NE entries (q = lo + l16 + 16 j; -1 past the end).
// Static during a solve, so the fused loops read it once.
template <int NE>
struct RowListN {
  int lo, hi, it[NE];
};
using RowList = RowListN<4>;

template <int NE = 4>
__device__ inline RowListN<NE> row_list(const int32_t* __restrict__ cam_ptr, const int32_t* __restrict__ cam_items,
                                        int c, int l16) {
  RowListN<NE> L;
  L.lo = cam_ptr[c];
  L.hi = cam_ptr[c + 1];
#pragma unroll
  for (int j = 0; j < NE; ++j) L.it[j] = L.lo + l16 + 16 * j < L.hi ? cam_items[L.lo + l16 + 16 * j] : -1;
  return L;
}

// A row list with no entries (rows past the last camera).
template <int NE = 4>
__device__ inline RowListN<NE> empty_row_list() {
  RowListN<NE> L;
  L.lo = L.hi = 0;
#pragma unroll
  for (int j = 0; j < NE; ++j) L.it[j] = -1;
  return L;
}

template <int CTRL>
__device__ inline double dpp_mov_d(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)bits, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Reduce-scatter stage over lane bit BIT (see the Gram pass for the partner
// rules): keep the lower or upper half of S values and add the partner's.
template <int S, int BIT>
__device__ inline void rs_stage_d(const double (&in)[S], double (&out)[(S + 1) / 2], int lane) {
  constexpr int H = (S + 1) / 2;
  const bool up = (lane >> BIT) & 1;
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const double lo = in[k];
    const double hi = (k + H < S) ? in[k + H] : 0.0;
    const double send = up ? lo : hi;
    double recv;
    if constexpr (BIT == 3) recv = dpp_mov_d<0x140>(send);        // row_mirror
    else if constexpr (BIT == 2) recv = dpp_mov_d<0x141>(send);   // row_half_mirror
    else if constexpr (BIT == 1) recv = dpp_mov_d<0x4E>(send);    // quad_perm xor 2
    else recv = dpp_mov_d<0xB1>(send);                            // quad_perm xor 1
    out[k] = (up ? hi : lo) + recv;
  }
}

// Adds one side (12 floats) of a pair record to acc.
__device__ inline void add_record(const float* __restrict__ contrib, int item, double acc[12]) {
  const float4* c = reinterpret_cast<const float4*>(contrib + (int64_t)(item >> 1) * 24 + (item & 1) * 12);
  const float4 r0 = c[0], r1 = c[1], r2 = c[2];
  acc[0] += r0.x; acc[1] += r0.y; acc[2] += r0.z; acc[3] += r0.w;
  acc[4] += r1.x; acc[5] += r1.y; acc[6] += r1.z; acc[7] += r1.w;
  acc[8] += r2.x; acc[9] += r2.y; acc[10] += r2.z; acc[11] += r2.w;
}

// Wave-wide total of the 12 per-lane sums (dL/dR 3x3, dL/dt), returned in
// every lane: reduce-scatter over lane bits 3..0 (12 -> 6 -> 3 -> 2 -> 1,
// DPP), add across the four rows, gather back.  Fixed order: deterministic.
__device__ inline void wave_sum12(double acc[12], int lane) {
  double b6[6], b3[3], b2[2], b1[1];
  rs_stage_d<12, 3>(*reinterpret_cast<double(*)[12]>(acc), b6, lane);
  rs_stage_d<6, 2>(b6, b3, lane);
  rs_stage_d<3, 1>(b3, b2, lane);
  rs_stage_d<2, 0>(b2, b1, lane);
  double v = b1[0];
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  // entry s now sits in lane s + s / 3 of every row
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = __shfl(v, k + k / 3);
}

// dL/dtheta [9] of one camera from its summed dL/dR (columns g1, g2, g3 in
// acc[3r + col]) and dL/dt (acc[9..11]): the Gram-Schmidt adjoint in float64.
__device__ inline void gs_adjoint(const double acc[12], const Gs& f, const double a2[3], double grad[9]) {
  double g1[3], g2[3], g3[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    g1[r] = acc[3 * r + 0];
    g2[r] = acc[3 * r + 1];
    g3[r] = acc[3 * r + 2];
  }
  // b3 = b1 x b2
  g1[0] += f.b2[1] * g3[2] - f.b2[2] * g3[1];
  g1[1] += f.b2[2] * g3[0] - f.b2[0] * g3[2];
  g1[2] += f.b2[0] * g3[1] - f.b2[1] * g3[0];
  g2[0] += g3[1] * f.b1[2] - g3[2] * f.b1[1];
  g2[1] += g3[2] * f.b1[0] - g3[0] * f.b1[2];
  g2[2] += g3[0] * f.b1[1] - g3[1] * f.b1[0];
  // b2 = u2/|u2|, u2 = a2 - (b1.a2) b1
  const double b2g2 = f.b2[0] * g2[0] + f.b2[1] * g2[1] + f.b2[2] * g2[2];
  double gu[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) gu[k] = (g2[k] - b2g2 * f.b2[k]) * f.r2;
  const double b1gu = f.b1[0] * gu[0] + f.b1[1] * gu[1] + f.b1[2] * gu[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    grad[3 + k] = gu[k] - f.b1[k] * b1gu;
    g1[k] += -f.d12 * gu[k] - a2[k] * b1gu;
  }
  // b1 = a1/|a1|
  const double b1g1 = f.b1[0] * g1[0] + f.b1[1] * g1[1] + f.b1[2] * g1[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    grad[k] = (g1[k] - b1g1 * f.b1[k]) * f.r1;
    grad[6 + k] = acc[9 + k];
  }
}

// The same from the parameters (the forward pass computed here).
__device__ inline void gs_adjoint(const double acc[12], const double a1[3], const double a2[3], double grad[9]) {
  gs_adjoint(acc, gs_forward(a1, a2), a2, grad);
}

// Row-wide total of the 12 per-lane sums over one 16-lane row, returned in
// every lane of the row: the same DPP reduce-scatter as wave_sum12 without
// the cross-row steps, then a gather inside the row.
__device__ inline void row_sum12(double acc[12], int lane) {
  double b6[6], b3[3], b2[2], b1[1];
  rs_stage_d<12, 3>(*reinterpret_cast<double(*)[12]>(acc), b6, lane);
  rs_stage_d<6, 2>(b6, b3, lane);
  rs_stage_d<3, 1>(b3, b2, lane);
  rs_stage_d<2, 0>(b2, b1, lane);
  const double v = b1[0];
  const int base = lane & ~15;
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = __shfl(v, base + k + k / 3);
}

// Summed records of one camera in every lane of its row.
__device__ inline void row_camera_sums(const RowList& L, const int32_t* __restrict__ cam_items,
                                       const float* __restrict__ contrib, int lane, double acc[12]) {
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (L.it[j] >= 0) add_record(contrib, L.it[j], acc);
  for (int q = L.lo + 64 + (lane & 15); q < L.hi; q += 16) add_record(contrib, cam_items[q], acc);
  row_sum12(acc, lane);
}

// Row-wide total of 6 per-lane sums over one 16-lane row, in every lane of
// the row: reduce-scatter over lane bits 3..1 (6 -> 3 -> 2 -> 1), the partner
// over bit 0 added, then a gather inside the row (entry s ends in lane
// 8 (s / 3) + 2 (s % 3) of the row).  Fixed order: deterministic.
__device__ inline double row_partial6(const double (&acc)[6], int lane) {
  double b3[3], b2[2], b1[1];
  rs_stage_d<6, 3>(acc, b3, lane);
  rs_stage_d<3, 2>(b3, b2, lane);
  rs_stage_d<2, 1>(b2, b1, lane);
  return b1[0] + dpp_mov_d<0xB1>(b1[0]);   // quad_perm xor 1
}

__device__ inline void row_sum6(double (&acc)[6], int lane) {
  const double v = row_partial6(acc, lane);
  const int base = lane & ~15;
#pragma unroll
  for (int k = 0; k < 6; ++k) acc[k] = __shfl(v, base + 8 * (k / 3) + 2 * (k % 3));
}

// Wave-wide total of 6 per-lane sums, in every lane: the row reduction, the
// four rows added, the gather.
__device__ inline void wave_sum6(double (&acc)[6], int lane) {
  double v = row_partial6(acc, lane);
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
#pragma unroll
  for (int k = 0; k < 6; ++k) acc[k] = __shfl(v, 8 * (k / 3) + 2 * (k % 3));
}

// A camera's summed body-frame rotation gradient om (sums of its pairs'
// essential_adjoint_omega terms) as dL/dR = R [om]_x, with R's columns
// b1, b2, b3 from its Gram-Schmidt, in the acc[12] layout gs_adjoint reads
// (dL/dR row-major, then dL/dt from dt).
__device__ inline void omega_grad(const Gs& f, const double om[3], const double dt[3], double acc[12]) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double R0 = f.b1[r], R1 = f.b2[r], R2 = f.b3[r];
    acc[3 * r + 0] = R1 * om[2] - R2 * om[1];
    acc[3 * r + 1] = R2 * om[0] - R0 * om[2];
    acc[3 * r + 2] = R0 * om[1] - R1 * om[0];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) acc[9 + k] = dt[k];
}

// The element q of a per-lane array held identically by all lanes.
__device__ inline double pick9(const double g[9], int q) {
  double v = g[0];
#pragma unroll
  for (int k = 1; k < 9; ++k) v = (q == k) ? g[k] : v;
  return v;
}

// Deterministic block sum of one double per thread (fixed tree).
__device__ inline double block_sum(double v, double* lds) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s);
  if (lane == 0) lds[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += lds[k];
  __syncthreads();
  return t;
}

// Step schedule of a persistent Adam loop: the learning-rate fraction
// exp(log_frac (lr_step0 + k) / lr_total) and the powers b1^s, b2^s of the
// bias corrections (s = adam_step0 + k + 1) for k = 0, 1, ..., evaluated
// with exp/pow at the launch's first step and then advanced by one product
// each per step (over a launch's steps the running products stay within
// ~1e-13 relative of the direct formulas; the direct ones cost two float64
// pow and an exp per lane per iteration).
struct StepSched {
  double frac, p1, p2;
  double dfrac, b1, b2;
  __device__ StepSched(double log_frac, int64_t lr_step0, int64_t lr_total, int64_t adam_step0, double b1_,
                       double b2_)
      : frac(exp(log_frac * (double)lr_step0 / (double)lr_total)),
        p1(pow(b1_, (double)(adam_step0 + 1))),
        p2(pow(b2_, (double)(adam_step0 + 1))),
        dfrac(exp(log_frac / (double)lr_total)),
        b1(b1_),
        b2(b2_) {}
  __device__ void next() {
    frac *= dfrac;
    p1 *= b1;
    p2 *= b2;
  }
};

// One Adam update (Kingma & Ba, bias-corrected) of a float32 value; the
// arithmetic is float64, the stored moments float32.  The bias corrections
// are applied as products with their reciprocals (uniform over a step, so
// the persistent loops compute them once per iteration).
__device__ inline float adam_update(float p, float g, float& m, float& v, double lr, double b1, double b2,
                                    double eps, double bc1, double bc2) {
  const double md = b1 * (double)m + (1.0 - b1) * (double)g;
  const double vd = b2 * (double)v + (1.0 - b2) * (double)g * (double)g;
  m = (float)md;
  v = (float)vd;
  const double ib1 = 1.0 / bc1, ib2 = 1.0 / bc2;
  return (float)((double)p - lr * (md * ib1) / (sqrt(vd * ib2) + eps));
}

// Pair count below which the epipolar persistent loop runs camera by camera
// when the caller leaves the grid automatic (the translation and rotation
// loops, whose pair terms are cheaper, always do): one wavefront
// per camera evaluates each of its pairs, so every pair is evaluated twice
// but an iteration needs one grid barrier and no record round trip.  Above
// it, where one wavefront per camera leaves the high-degree cameras'
// wavefronts long and the rest idle, the pair loop wins.  Measured with the
// epipolar loop, float64 Grams, per iteration (camera vs pair loop): 200
// cameras / 4.9k pairs 10.5 vs 16.1 us; banded graphs 1,000 / 24.7k 12.3 vs
// 33.4, 2,500 / 124k 34.3 vs 39.9, 5,000 / 249k 47.1 vs 50.7; the 5,000-camera
// street graph (185k pairs, uneven degrees) 44.3 vs 41.0.
constexpr int64_t kCamLoopMaxPairs = 131072;

// Workgroup count from which the fused epipolar loops synchronise with the
// per-XCD grid_sync instead of the flat grid_barrier.  Per iteration, flat
// vs per-XCD: large street graph, pair loop at 192 workgroups 37.0 vs
// 29.2 us; camera loop at 256 workgroups 38.2 vs 35.9 us; medium helix
// scene, camera loop at 25 workgroups 9.75 vs 11.15 us, pair loop at 16 and
// 64 workgroups 14.9 vs 17.2 and 15.5 vs 17.3 us (the second level of
// notification costs more than the fences it saves on small grids).
constexpr int64_t kXcdSyncMinBlocks = 128;

constexpr unsigned kBarSpinOuter = 1u << 14;   // x 256 polls
// XCD slots of the grid_sync barrier (the XCC_ID hardware field is 4 bits).
constexpr int kMaxXcd = 16;
// Words of `bar`, one 128-byte line each: arrival count and generation of
// grid_barrier (words 0 and 32), failure flag of the running launch (64),
// failure total since the last query (96); then per XCD the arrival count
// and generation of grid_sync and the number of the launch's workgroups on
// that XCD; then grid_sync's count of XCDs arrived.  Every count and generation starts the
// launch at 0 (fm_bar_reset) and only grows, so a workgroup knows the value
// at which each barrier opens without reading anything first.
constexpr int kBarXcdCount = 128;
constexpr int kBarXcdGen = kBarXcdCount + 32 * kMaxXcd;
constexpr int kBarXcdReg = kBarXcdGen + 32 * kMaxXcd;
constexpr int kBarTop = kBarXcdReg + 32 * kMaxXcd;
constexpr int kBarWords = kBarTop + 32;

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their maxima)
constexpr int kWaitVmcnt0 = 0x0F70;

__device__ inline unsigned bar_load(unsigned* w) {
  return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait of thread 0 until the count w reaches `target` (compared
// modulo 2^32: a waiter is never more than one barrier behind).  If the wait
// expires (the workgroups were not all resident) or another workgroup has
// raised the launch's failure flag, it raises the flag and the scene's
// failure total; every later barrier of the launch then returns at once and
// the host reads the total with fm_solve_barrier_failures.
__device__ inline void bar_reach(unsigned* __restrict__ bar, unsigned* w, unsigned target) {
  unsigned* fail = bar + 64;
  bool reached = false;
  for (unsigned outer = 0; outer < kBarSpinOuter && !reached; ++outer) {
#pragma unroll 1
    for (int i = 0; i < 256; ++i) {
      if ((int)(bar_load(w) - target) >= 0) {
        reached = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (!reached && bar_load(fail) != 0u) break;
  }
  if (!reached) {
    __hip_atomic_fetch_add(fail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(bar + 96, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One workgroup's state of the flat grid barrier (the same in every thread):
// the arrival count and the generation at which the launch's next barrier
// opens.
struct GridBar {
  unsigned* bar;
  unsigned next, gnext;
};

__device__ inline GridBar grid_bar(unsigned* bar) { return GridBar{bar, gridDim.x, 1u}; }

// Store at agent scope (relaxed atomic): written through to memory, so it is
// visible on every XCD once complete, with no L2 write-back.
template <typename T>
__device__ inline void store_wt(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Flat grid barrier of the persistent loops.  Thread 0 of each workgroup
// makes the workgroup's writes visible and counts itself in; the workgroup
// whose increment brings the count to the barrier's opening value stores
// the new generation, which the others wait for (polling a word that no
// arrival increments); each then acquires (invalidates its XCD's L2 and its
// CU's L1).  Counts and generations are never reset within a launch, so a
// workgroup knows both opening values without reading anything first, and
// opening the barrier takes one store.  That store needs no fence of its
// own: every workgroup's writes reached memory before its increment, and
// the store is issued only after the last increment has returned.  All
// atomics are relaxed and agent-scoped; the fences carry the ordering.  The
// failure flag is read before the workgroup gathers, so that its latency
// overlaps the wait for the other wavefronts.
//
// Making the writes visible: with WT false (data shared through plain
// stores) an agent-scope release, which writes back the dirty lines of the
// XCD's L2; with WT true (everything other workgroups read after the
// barrier was written with store_wt) only each thread's wait for its own
// stores to complete, so no L2 write-back sits on the path of the last
// workgroup to arrive.  Data a workgroup alone reads back (its own Adam
// moments) may still be written with plain stores.
template <bool WT>
__device__ inline void grid_barrier_t(GridBar& gb) {
  unsigned* count = gb.bar;
  unsigned* gen = gb.bar + 32;
  unsigned f = 0u;
  if (threadIdx.x == 0) f = bar_load(gb.bar + 64);
  if constexpr (WT) __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  __syncthreads();
  if (threadIdx.x == 0 && f == 0u) {
    if constexpr (!WT) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (__hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u == gb.next)
      __hip_atomic_store(gen, gb.gnext, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      bar_reach(gb.bar, gen, gb.gnext);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  gb.next += gridDim.x;
  gb.gnext += 1u;
  __syncthreads();
}

__device__ inline void grid_barrier(GridBar& gb) { grid_barrier_t<false>(gb); }
__device__ inline void grid_barrier_wt(GridBar& gb) { grid_barrier_t<true>(gb); }

// XCD of the running workgroup (hardware register XCC_ID, bits 3:0), and
// after xcd_register the number of the launch's workgroups on it, the number
// of XCDs that hold any, and the opening values of the next grid_sync: the
// XCD's arrival count, the count of XCDs arrived, and the XCD's generation.
struct XcdSync {
  unsigned x, nx, nact;
  unsigned lnext, tnext, gnext;
};

__device__ inline unsigned xcc_id() {
  // s_getreg_b32 hwreg(HW_REG_XCC_ID = 20, offset 0, size 4)
  return (unsigned)__builtin_amdgcn_s_getreg(20 | (3 << 11)) & (kMaxXcd - 1);
}

// Called once by every thread at the start of a launch that uses grid_sync
// (the counters were cleared by fm_bar_reset); ends with a grid_barrier on gb.
__device__ inline XcdSync xcd_register(GridBar& gb) {
  XcdSync xs;
  xs.x = xcc_id();
  if (threadIdx.x == 0)
    __hip_atomic_fetch_add(gb.bar + kBarXcdReg + 32 * xs.x, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  grid_barrier(gb);
  xs.nx = 0;
  xs.nact = 0;
  for (int k = 0; k < kMaxXcd; ++k) {
    const unsigned n = bar_load(gb.bar + kBarXcdReg + 32 * k);
    if ((unsigned)k == xs.x) xs.nx = n;
    xs.nact += n > 0u ? 1u : 0u;
  }
  xs.lnext = xs.nx;
  xs.tnext = xs.nact;
  xs.gnext = 1u;
  return xs;
}

// Grid barrier for loops whose data shared between workgroups is written
// with plain stores.  The L2 write-back runs once per XCD instead of once
// per workgroup: each thread waits for its own stores to reach the L2; the
// workgroups of an XCD count in on the XCD's counter; the last of them
// writes the XCD's L2 back (agent-scope release), counts the XCD in on the
// top-level counter and waits for every XCD to have arrived, invalidates the
// XCD's L2 (agent-scope acquire; complete before it moves on) and moves the
// XCD's generation word, which the XCD's other workgroups wait for.  Each of
// those then acquires too: that invalidates its CU's L1, which may still hold
// lines it read before the barrier (loads of group scope, sc0, are served
// from the L1 as plain ones are, and an L1 invalidation of group scope does
// nothing in a workgroup that is not split across CUs; only the agent-scope
// invalidation clears it).  As in grid_barrier, counts and generations only
// grow within a launch.
__device__ inline void grid_sync(unsigned* __restrict__ bar, XcdSync& xs) {
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  unsigned f = 0u;
  if (threadIdx.x == 0) f = bar_load(bar + 64);
  __syncthreads();
  if (threadIdx.x == 0 && f == 0u) {
    unsigned* xc = bar + kBarXcdCount + 32 * xs.x;
    unsigned* xg = bar + kBarXcdGen + 32 * xs.x;
    if (__hip_atomic_fetch_add(xc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u == xs.lnext) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      unsigned* top = bar + kBarTop;
      if (__hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u != xs.tnext)
        bar_reach(bar, top, xs.tnext);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
      __hip_atomic_store(xg, xs.gnext, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      bar_reach(bar, xg, xs.gnext);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  xs.lnext += xs.nx;
  xs.tnext += xs.nact;
  xs.gnext += 1u;
  __syncthreads();
}

// Clears the counts, generations and registrations of the grid barriers and
// the launch's failure flag before a persistent launch (iterate.hip); every
// launch that uses grid_barrier or grid_sync needs it.
hipError_t fm_bar_reset(unsigned* bar, hipStream_t st);
