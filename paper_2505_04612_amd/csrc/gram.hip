// Per-pair Gram build (App. B.6) and IRLS reweighting (Sec. 3.3).
//
// The M matches are streamed once, in pair order.  Work item w covers up to
// kChunk = 1024 consecutive matches of one pair and is processed by one
// wavefront: lane l takes matches start + l + 64 r (so every load instruction
// of the wave reads one contiguous span), forms the monomials
// p = (u^2, uv, v^2, u, v, 1) of both points and accumulates the 36 sums
// omega p2[q2] p1[q1] in float32 registers.  A reduce-scatter across the wave
// (38 lane exchanges instead of 36 full reductions) leaves one entry per lane
// in 36 of the 64 lanes, which store the work item's partial Gram.  A second
// kernel adds each pair's partials in float64, in work-item order, so the
// result does not depend on scheduling: no atomics touch floating point.
#include "fm_internal.h"

enum { W_UNIT = 0, W_ARRAY = 1, W_IRLS = 2 };

template <int DT>
__device__ inline float4 load_match(const void* uv, int64_t m) {
  if constexpr (DT == FM_F32) {
    return reinterpret_cast<const float4*>(uv)[m];
  } else if constexpr (DT == FM_BF16) {
    // four bf16 values: the float32 with the same upper 16 bits
    uint2 q = reinterpret_cast<const uint2*>(uv)[m];
    return make_float4(__uint_as_float(q.x << 16), __uint_as_float(q.x & 0xffff0000u),
                       __uint_as_float(q.y << 16), __uint_as_float(q.y & 0xffff0000u));
  } else {
    const double2* d = reinterpret_cast<const double2*>(uv) + 2 * m;
    double2 a = d[0], b = d[1];
    return make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
  }
}

// The exact float64 value of the stored coordinates (used for the residual).
template <int DT>
__device__ inline void load_match_f64(const void* uv, int64_t m, float4 f, double x[4]) {
  if constexpr (DT == FM_F64) {
    const double2* d = reinterpret_cast<const double2*>(uv) + 2 * m;
    double2 a = d[0], b = d[1];
    x[0] = a.x; x[1] = a.y; x[2] = b.x; x[3] = b.y;
  } else {
    x[0] = f.x; x[1] = f.y; x[2] = f.z; x[3] = f.w;
  }
}

// Reduce-scatter of 36 per-lane values over the 64 lanes of a wavefront.
// Stage k exchanges half of the current values with the lane whose index
// differs in bit (5 - k) and keeps the other half (padded to an even count);
// after six stages each lane holds the wave total of at most one entry.
// Returns that total; `slot` receives the entry index or -1.
__device__ inline float wave_reduce_scatter36(const float (&a)[36], int lane, int& slot) {
  float b[18], c[9], d[5], e[3], f[2];
  bool up = (lane & 32) != 0;
#pragma unroll
  for (int k = 0; k < 18; ++k) {
    float send = up ? a[k] : a[k + 18];
    float keep = up ? a[k + 18] : a[k];
    b[k] = keep + __shfl_xor(send, 32);
  }
  up = (lane & 16) != 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    float send = up ? b[k] : b[k + 9];
    float keep = up ? b[k + 9] : b[k];
    c[k] = keep + __shfl_xor(send, 16);
  }
  up = (lane & 8) != 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    float hi = (k + 5 < 9) ? c[k + 5] : 0.0f;
    float send = up ? c[k] : hi;
    float keep = up ? hi : c[k];
    d[k] = keep + __shfl_xor(send, 8);
  }
  up = (lane & 4) != 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float hi = (k + 3 < 5) ? d[k + 3] : 0.0f;
    float send = up ? d[k] : hi;
    float keep = up ? hi : d[k];
    e[k] = keep + __shfl_xor(send, 4);
  }
  up = (lane & 2) != 0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    float hi = (k + 2 < 3) ? e[k + 2] : 0.0f;
    float send = up ? e[k] : hi;
    float keep = up ? hi : e[k];
    f[k] = keep + __shfl_xor(send, 2);
  }
  up = (lane & 1) != 0;
  float g = (up ? f[1] : f[0]) + __shfl_xor(up ? f[0] : f[1], 1);
  // entry index held by this lane (see the stage sizes 36, 18, 9, 5, 3, 2)
  int x = lane & 1;
  int y = x + 2 * ((lane >> 1) & 1);
  int z = y + 3 * ((lane >> 2) & 1);
  int w = z + 5 * ((lane >> 3) & 1);
  slot = (y < 3 && z < 5 && w < 9) ? w + 9 * ((lane >> 4) & 1) + 18 * ((lane >> 5) & 1) : -1;
  return g;
}

__device__ inline int64_t find_pair(const int64_t* wi_off, int64_t P, int64_t w) {
  // largest n with wi_off[n] <= w; wi_off[0] = 0 <= w < wi_off[P]
  int64_t lo = 0, hi = P;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (wi_off[mid] <= w) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ inline void accumulate36(float (&acc)[36], float4 x, float om) {
  // p1 = monomials of x1 = (u1, v1), p2 of x2 = (u2, v2)
  const float p1[5] = {x.x * x.x, x.x * x.y, x.y * x.y, x.x, x.y};
  const float w2[6] = {om * (x.z * x.z), om * (x.z * x.w), om * (x.w * x.w), om * x.z, om * x.w, om};
#pragma unroll
  for (int q2 = 0; q2 < 6; ++q2) {
#pragma unroll
    for (int q1 = 0; q1 < 5; ++q1) acc[6 * q2 + q1] = fmaf(w2[q2], p1[q1], acc[6 * q2 + q1]);
    acc[6 * q2 + 5] += w2[q2];
  }
}

// One wavefront per work item.  WMODE: W_UNIT (omega = 1), W_ARRAY (omega from
// `weights`) or W_IRLS (omega from the residual at E_n).  BUILD: accumulate the
// Gram partials.  WRITE: store omega (and r if r_out) per match.
template <int DT, int WMODE, bool BUILD, bool WRITE>
__global__ __launch_bounds__(kGramWaves * kLanes) void k_gram_partial(
    const void* __restrict__ uv, const int64_t* __restrict__ off, const int64_t* __restrict__ wi_off,
    int64_t P, int64_t n_wi, const float* __restrict__ weights, const double* __restrict__ ess,
    double delta, double tau, float* __restrict__ partials, float* __restrict__ w_out,
    float* __restrict__ r_out, unsigned long long* __restrict__ kept) {
  const int lane = threadIdx.x & (kLanes - 1);
  const int64_t w = (int64_t)blockIdx.x * kGramWaves + (threadIdx.x >> 6);
  if (w >= n_wi) return;  // whole wavefront
  const int64_t n = find_pair(wi_off, P, w);
  const int64_t start = off[n] + (w - wi_off[n]) * kChunk;
  const int64_t stop = min(off[n + 1], start + kChunk);
  const int count = (int)(stop - start);
  double E[9];
  if constexpr (WMODE == W_IRLS) {
#pragma unroll
    for (int k = 0; k < 9; ++k) E[k] = ess[n * 9 + k];
  }
  float acc[36];
#pragma unroll
  for (int k = 0; k < 36; ++k) acc[k] = 0.0f;
  unsigned nkept = 0;
  // groups of 4 matches per lane; the group loop exits uniformly
#pragma unroll
  for (int g = 0; g < kPerLane / 4; ++g) {
    if (g * 4 * kLanes >= count) break;
    // lanes past the end of the chunk load the chunk's first match (always
    // in bounds) and get weight 0
    float4 xs[4];
    bool ok[4];
    int64_t mi[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = (g * 4 + r) * kLanes + lane;
      ok[r] = i < count;
      mi[r] = ok[r] ? start + i : start;
      xs[r] = load_match<DT>(uv, mi[r]);
    }
    float oms[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = mi[r];
      float om = ok[r] ? 1.0f : 0.0f;
      if constexpr (WMODE == W_ARRAY) {
        const float wm = weights[m];
        om = ok[r] ? wm : 0.0f;
      } else if constexpr (WMODE == W_IRLS) {
        // r = x2~^T E x1~ in float64 from the stored coordinates
        double x[4];
        load_match_f64<DT>(uv, m, xs[r], x);
        const double e0 = E[0] * x[0] + E[1] * x[1] + E[2];
        const double e1 = E[3] * x[0] + E[4] * x[1] + E[5];
        const double e2 = E[6] * x[0] + E[7] * x[1] + E[8];
        const double res = x[2] * e0 + x[3] * e1 + e2;
        const double a = fabs(res);
        om = (ok[r] && a <= tau) ? (float)(1.0 / (a > delta ? a : delta)) : 0.0f;
        nkept += (om > 0.0f) ? 1u : 0u;
        if constexpr (WRITE) {
          if (ok[r] && r_out) r_out[m] = (float)res;
        }
      }
      if constexpr (WRITE) {
        if (ok[r]) w_out[m] = om;
      }
      oms[r] = om;
    }
    if constexpr (BUILD) {
#pragma unroll
      for (int r = 0; r < 4; ++r) accumulate36(acc, xs[r], oms[r]);
    }
  }
  if constexpr (BUILD) {
    int slot;
    const float v = wave_reduce_scatter36(acc, lane, slot);
    if (slot >= 0) partials[w * 36 + slot] = v;
  }
  if constexpr (WMODE == W_IRLS) {
    // integer wave sum, one atomic per wavefront (exact, order-free)
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) nkept += __shfl_xor(nkept, s);
    if (lane == 0 && nkept) atomicAdd(kept, (unsigned long long)nkept);
  }
}

// Sum each pair's work-item partials in float64, in work-item order.
__global__ void k_gram_finalize(const float* __restrict__ partials, const int64_t* __restrict__ wi_off,
                                int64_t P, double* __restrict__ W64, float* __restrict__ W32) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P * 36) return;
  const int64_t n = t / 36;
  const int k = (int)(t - n * 36);
  double s = 0.0;
  for (int64_t w = wi_off[n]; w < wi_off[n + 1]; ++w) s += (double)partials[w * 36 + k];
  if (W64) W64[t] = s;
  if (W32) W32[t] = (float)s;
}

// E_n for every pair at the given poses (float64), for the residual pass;
// thread 0 also clears the kept-match counter.
__global__ void k_pair_essentials(const float* __restrict__ params, const int32_t* __restrict__ cams,
                                  int64_t P, double* __restrict__ ess, unsigned long long* kept) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n == 0 && kept) *kept = 0ull;
  if (n >= P) return;
  double a1[3], a2[3], ti[3], tj[3];
  double Ri[3][3], Rj[3][3], Rij[3][3], th[3], E[3][3];
  load_pose(params, cams[2 * n], a1, a2, ti);
  gs_matrix(gs_forward(a1, a2), Ri);
  load_pose(params, cams[2 * n + 1], a1, a2, tj);
  gs_matrix(gs_forward(a1, a2), Rj);
  pair_essential(Ri, ti, Rj, tj, Rij, th, E);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) ess[n * 9 + 3 * a + b] = E[a][b];
}

// ------------------------------------------------------------------ host side

template <int WMODE, bool BUILD, bool WRITE>
static fm_status launch_partial(fm_scene* s, const float* weights, double delta, double tau, float* w_out,
                                float* r_out, unsigned long long* kept, hipStream_t st) {
  if (s->n_wi == 0) return FM_OK;
  const dim3 grid(grid_for(s->n_wi, kGramWaves)), block(kGramWaves * kLanes);
  fm_timed timer(s->ctx, FM_K_GRAM, st);
  switch (s->dtype) {
    case FM_F32:
      hipLaunchKernelGGL((k_gram_partial<FM_F32, WMODE, BUILD, WRITE>), grid, block, 0, st, s->uv, s->offsets,
                         s->wi_off, s->P, s->n_wi, weights, s->ess, delta, tau, s->partials, w_out, r_out, kept);
      break;
    case FM_BF16:
      hipLaunchKernelGGL((k_gram_partial<FM_BF16, WMODE, BUILD, WRITE>), grid, block, 0, st, s->uv, s->offsets,
                         s->wi_off, s->P, s->n_wi, weights, s->ess, delta, tau, s->partials, w_out, r_out, kept);
      break;
    default:
      hipLaunchKernelGGL((k_gram_partial<FM_F64, WMODE, BUILD, WRITE>), grid, block, 0, st, s->uv, s->offsets,
                         s->wi_off, s->P, s->n_wi, weights, s->ess, delta, tau, s->partials, w_out, r_out, kept);
      break;
  }
  FM_CHECK_LAUNCH(s->ctx);
  return FM_OK;
}

static fm_status launch_finalize(fm_scene* s, double* W64, float* W32, hipStream_t st) {
  if (s->P == 0) return FM_OK;
  fm_timed timer(s->ctx, FM_K_FINALIZE, st);
  hipLaunchKernelGGL(k_gram_finalize, dim3(grid_for(s->P * 36, kBlock)), dim3(kBlock), 0, st, s->partials,
                     s->wi_off, s->P, W64, W32);
  FM_CHECK_LAUNCH(s->ctx);
  return FM_OK;
}

static fm_status launch_essentials(fm_scene* s, const float* params, unsigned long long* kept, hipStream_t st) {
  fm_timed timer(s->ctx, FM_K_ESSENTIALS, st);
  hipLaunchKernelGGL(k_pair_essentials, dim3(grid_for(s->P > 0 ? s->P : 1, kBlock)), dim3(kBlock), 0, st, params,
                     s->pair_cams, s->P, s->ess, kept);
  FM_CHECK_LAUNCH(s->ctx);
  return FM_OK;
}

fm_status fm_launch_essentials(fm_scene* s, const float* params, unsigned long long* kept, hipStream_t st) {
  return launch_essentials(s, params, kept, st);
}

static fm_status check_scene(fm_ctx* ctx, fm_scene* s, const char* fn) {
  if (!ctx) return FM_EINVAL;
  if (!s) return fm_fail(ctx, FM_EINVAL, "%s: scene is NULL", fn);
  if (s->ctx != ctx) return fm_fail(ctx, FM_EINVAL, "%s: scene belongs to another context", fn);
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  return FM_OK;
}

extern "C" fm_status fm_build_pair_grams(fm_ctx* ctx, fm_scene* s, const float* weights, double* W64,
                                         float* W32, fm_stream stream) {
  fm_status rc = check_scene(ctx, s, "fm_build_pair_grams");
  if (rc != FM_OK) return rc;
  if (!W64 && !W32 && s->P > 0) return fm_fail(ctx, FM_EINVAL, "fm_build_pair_grams: both outputs are NULL");
  hipStream_t st = (hipStream_t)stream;
  rc = weights ? launch_partial<W_ARRAY, true, false>(s, weights, 0, 0, nullptr, nullptr, nullptr, st)
               : launch_partial<W_UNIT, true, false>(s, nullptr, 0, 0, nullptr, nullptr, nullptr, st);
  if (rc != FM_OK) return rc;
  return launch_finalize(s, W64, W32, st);
}

static fm_status check_irls_args(fm_ctx* ctx, const char* fn, const float* params, float delta, float tau,
                                 int64_t* kept) {
  if (!params) return fm_fail(ctx, FM_EINVAL, "%s: params is NULL", fn);
  if (!kept) return fm_fail(ctx, FM_EINVAL, "%s: num_kept is NULL", fn);
  if (!(delta > 0.0f) || !(tau > 0.0f)) return fm_fail(ctx, FM_EINVAL, "%s: delta and tau must be > 0", fn);
  return FM_OK;
}

extern "C" fm_status fm_reweight(fm_ctx* ctx, fm_scene* s, const float* params, float delta, float tau,
                                 float* w_out, float* r_out, int64_t* kept, fm_stream stream) {
  fm_status rc = check_scene(ctx, s, "fm_reweight");
  if (rc != FM_OK) return rc;
  if ((rc = check_irls_args(ctx, "fm_reweight", params, delta, tau, kept)) != FM_OK) return rc;
  if (!w_out && s->M > 0) return fm_fail(ctx, FM_EINVAL, "fm_reweight: weights_out is NULL");
  hipStream_t st = (hipStream_t)stream;
  unsigned long long* k = reinterpret_cast<unsigned long long*>(kept);
  if ((rc = launch_essentials(s, params, k, st)) != FM_OK) return rc;
  return launch_partial<W_IRLS, false, true>(s, nullptr, delta, tau, w_out, r_out, k, st);
}

extern "C" fm_status fm_reweight_build(fm_ctx* ctx, fm_scene* s, const float* params, float delta, float tau,
                                       double* W64, float* W32, int64_t* kept, fm_stream stream) {
  fm_status rc = check_scene(ctx, s, "fm_reweight_build");
  if (rc != FM_OK) return rc;
  if ((rc = check_irls_args(ctx, "fm_reweight_build", params, delta, tau, kept)) != FM_OK) return rc;
  if (!W64 && !W32 && s->P > 0) return fm_fail(ctx, FM_EINVAL, "fm_reweight_build: both outputs are NULL");
  hipStream_t st = (hipStream_t)stream;
  unsigned long long* k = reinterpret_cast<unsigned long long*>(kept);
  if ((rc = launch_essentials(s, params, k, st)) != FM_OK) return rc;
  if ((rc = launch_partial<W_IRLS, true, false>(s, nullptr, delta, tau, nullptr, nullptr, k, st)) != FM_OK)
    return rc;
  return launch_finalize(s, W64, W32, st);
}
