// Per-pair Gram build (App. B.6) and IRLS reweighting (Sec. 3.3).
//
// The M matches are streamed once.  A work item is either a chunk of up to
// 1024 (BF16: 4096) consecutive matches of one pair, processed by a whole
// wavefront (lane l takes matches start + l + 64 r, so every load
// instruction of the wave reads one contiguous span), or four pairs of at
// most 256 (BF16: 1024) matches, 16 lanes each.  Each lane forms the
// monomials p = (u^2, uv, v^2, u, v, 1) of both points and accumulates the
// 36 sums omega p2[q2] p1[q1] in float32 registers; a reduce-scatter across
// the lanes of the pair (DPP and lane permutes: 38 exchanges instead of 36
// full reductions over a wavefront) leaves one entry per lane.  A pair that
// one work item covers stores its Gram directly; the chunks of a larger pair
// leave partials that a second kernel adds in float64, in chunk order, so the
// result does not depend on scheduling: no atomics touch floating point.
// (Adding them in the pass itself, by whichever chunk of a pair finishes
// last, needs an agent-scope release per chunk, and on this GPU each such
// release writes back the whole L2 of the chunk's XCD: measured 5-6x slower.)
#include "fm_internal.h"

enum { W_UNIT = 0, W_ARRAY = 1, W_IRLS = 2 };

// Lane exchange partners for the reduce-scatter.  Stages over lane bits 3,
// 2, 1, 0 use DPP within 16-lane rows (row_mirror pairs l with 15-l,
// row_half_mirror pairs l with 7-l inside each half row, quad_perm swaps
// neighbours 2 and 1 apart); bits 4 and 5 cross rows and use a lane
// permute.  Each pairing is an involution whose partner has the opposite
// value of the stage's bit and the same value of every bit already reduced,
// which is all a reduce-scatter needs.
template <int CTRL>
__device__ inline float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
constexpr int kDppRowMirror = 0x140, kDppHalfMirror = 0x141, kDppXor2 = 0x4E, kDppXor1 = 0xB1;

template <int S, int BIT>
__device__ inline float partner(float v) {
  if constexpr (BIT == 3) return dpp_mov<kDppRowMirror>(v);
  else if constexpr (BIT == 2) return dpp_mov<kDppHalfMirror>(v);
  else if constexpr (BIT == 1) return dpp_mov<kDppXor2>(v);
  else if constexpr (BIT == 0) return dpp_mov<kDppXor1>(v);
  else return __shfl_xor(v, 1 << BIT);
}

// One stage: keep the lower (bit clear) or upper (bit set) half of S values,
// padded to an even count, and add the partner's copy of that half.
template <int S, int BIT>
__device__ inline void rs_stage(const float (&in)[S], float (&out)[(S + 1) / 2], int lane) {
  constexpr int H = (S + 1) / 2;
  const bool up = (lane >> BIT) & 1;
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const float lo = in[k];
    const float hi = (k + H < S) ? in[k + H] : 0.0f;
    out[k] = (up ? hi : lo) + partner<S, BIT>(up ? lo : hi);
  }
}

// Reduce-scatter of 36 per-lane values over the 64 lanes of a wavefront
// (36 -> 18 -> 9 -> 5 -> 3 -> 2 -> 1 values per lane over lane bits 3, 2, 1,
// 0, 4, 5); afterwards 36 of the 64 lanes each hold the wave total of one
// entry.  Returns that total; `slot` receives the entry index or -1.
__device__ inline float wave_reduce_scatter36(const float (&a)[36], int lane, int& slot) {
  float b[18], c[9], d[5], e[3], f[2], g[1];
  rs_stage<36, 3>(a, b, lane);
  rs_stage<18, 2>(b, c, lane);
  rs_stage<9, 1>(c, d, lane);
  rs_stage<5, 0>(d, e, lane);
  rs_stage<3, 4>(e, f, lane);
  rs_stage<2, 5>(f, g, lane);
  // position of the kept value, walking the stages backwards
  const int b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
  const int b4 = (lane >> 4) & 1, b5 = (lane >> 5) & 1;
  const int x = b5;               // in the 2 values of stage 5
  const int y = x + 2 * b4;       // in the 3 values of stage 4
  const int z = y + 3 * b0;       // in the 5 values of stage 3
  const int w = z + 5 * b1;       // in the 9 values of stage 2
  slot = (y < 3 && z < 5 && w < 9) ? w + 9 * b2 + 18 * b3 : -1;
  return g[0];
}

__device__ inline void accumulate36(float (&acc)[36], float4 x, float om) {
  // p1 = monomials of x1 = (u1, v1); w2 = omega times the monomials of x2
  const float p1[5] = {x.x * x.x, x.x * x.y, x.y * x.y, x.x, x.y};
  const float ou = om * x.z, ov = om * x.w;
  const float w2[6] = {ou * x.z, ou * x.w, ov * x.w, ou, ov, om};
#pragma unroll
  for (int q2 = 0; q2 < 6; ++q2) {
#pragma unroll
    for (int q1 = 0; q1 < 5; ++q1) acc[6 * q2 + q1] = fmaf(w2[q2], p1[q1], acc[6 * q2 + q1]);
    acc[6 * q2 + 5] += w2[q2];
  }
}

// Raw storage of one match row per lane.
template <int DT> struct RawMatch;
template <> struct RawMatch<FM_F32> { using T = float4; };
template <> struct RawMatch<FM_BF16> { using T = uint2; };
template <> struct RawMatch<FM_F64> { using T = double4; };

template <int DT>
__device__ inline typename RawMatch<DT>::T load_raw(const typename RawMatch<DT>::T* __restrict__ p) {
  if constexpr (DT == FM_F64) {
    const double2* d = reinterpret_cast<const double2*>(p);
    const double2 a = d[0], b = d[1];
    return double4{a.x, a.y, b.x, b.y};
  } else {
    return *p;
  }
}

template <int DT>
__device__ inline void unpack(const typename RawMatch<DT>::T& r, float4& f, double x[4]) {
  if constexpr (DT == FM_F32) {
    f = r;
  } else if constexpr (DT == FM_BF16) {
    // bf16 -> the float32 with the same upper 16 bits
    f = make_float4(__uint_as_float(r.x << 16), __uint_as_float(r.x & 0xffff0000u),
                    __uint_as_float(r.y << 16), __uint_as_float(r.y & 0xffff0000u));
  } else {
    f = make_float4((float)r.x, (float)r.y, (float)r.z, (float)r.w);
  }
  if constexpr (DT == FM_F64) {
    x[0] = r.x; x[1] = r.y; x[2] = r.z; x[3] = r.w;
  } else {
    x[0] = f.x; x[1] = f.y; x[2] = f.z; x[3] = f.w;
  }
}

// Weight of one match and its contribution to the accumulators.  WMODE:
// W_UNIT (omega = 1), W_ARRAY (omega from `weights`) or W_IRLS (omega from
// the float64 residual at E_n).  BUILD: accumulate the Gram sums.  WRITE:
// store omega (and r if r_out).  CHECKED: `ok` says whether this lane's row
// entry is a match of the work item (lanes past the end carry weight 0);
// unchecked rows are full.  The kept count of an IRLS pass is taken per
// wavefront with a ballot, so it lives in a scalar register.
template <int DT, int WMODE, bool BUILD, bool WRITE, bool CHECKED>
__device__ inline void process_match(const typename RawMatch<DT>::T& raw, bool ok, int64_t m, const double E[9],
                                     float fdelta, double tau, const float* __restrict__ weights,
                                     float* __restrict__ w_out, float* __restrict__ r_out, float (&acc)[36],
                                     unsigned& nkept) {
  float4 xf;
  double x[4];
  unpack<DT>(raw, xf, x);
  float om = 1.0f;
  if constexpr (WMODE == W_UNIT) {
    if constexpr (CHECKED) om = ok ? 1.0f : 0.0f;
  } else if constexpr (WMODE == W_ARRAY) {
    om = weights[m];
    if constexpr (CHECKED) om = ok ? om : 0.0f;
  } else {
    // r = x2~^T E x1~ in float64 from the stored coordinates; the
    // keep/filter decision is taken on that value
    const double e0 = fma(E[0], x[0], fma(E[1], x[1], E[2]));
    const double e1 = fma(E[3], x[0], fma(E[4], x[1], E[5]));
    const double e2 = fma(E[6], x[0], fma(E[7], x[1], E[8]));
    const double res = fma(x[2], e0, fma(x[3], e1, e2));
    const double a = fabs(res);
    bool keep = a <= tau;
    if constexpr (CHECKED) keep = keep && ok;
    const float af = fmaxf((float)a, fdelta);
    om = keep ? __builtin_amdgcn_rcpf(af) : 0.0f;
    nkept += (unsigned)__popcll(__ballot(keep));
    if constexpr (WRITE) {
      if (r_out && (!CHECKED || ok)) r_out[m] = (float)res;
    }
  }
  if constexpr (WRITE) {
    if (!CHECKED || ok) w_out[m] = om;
  }
  if constexpr (BUILD) accumulate36(acc, xf, om);
}

// Stream the rows of one work item: this lane takes matches
// start + lid + STRIDE r for r < nrows <= ROWS (nrows is the same in every
// lane of the wavefront).  Rows below `nfull` are full and load straight from a
// per-lane pointer; the rows from nfull on are checked against `count`
// (lanes past it load the item's first match and weigh it 0).  Full rows are
// loaded BATCH at a time before any is used; a single checked row is loaded
// with the first batch.
template <int DT, int WMODE, bool BUILD, bool WRITE, int STRIDE, int BATCH, int ROWS>
__device__ inline void stream_rows(const void* __restrict__ uv, int64_t start, int count, int lid, int nrows,
                                   int nfull, const double E[9], float fdelta, double tau,
                                   const float* __restrict__ weights, float* __restrict__ w_out,
                                   float* __restrict__ r_out, float (&acc)[36], unsigned& nkept) {
  using RawT = typename RawMatch<DT>::T;
  const RawT* __restrict__ base = reinterpret_cast<const RawT*>(uv) + start;
  const RawT* __restrict__ p = base + lid;
  const int64_t m0 = start + lid;
  const bool one_tail = nrows - nfull == 1;
  RawT traw;
  const int ti = nfull * STRIDE + lid;
  const bool tok = ti < count;
  if (one_tail) traw = load_raw<DT>(tok ? p + nfull * STRIDE : base);
#pragma unroll
  for (int r0 = 0; r0 < ROWS; r0 += BATCH) {
    if (r0 < nfull) {
      RawT raw[BATCH];
      // one base per 8 rows keeps every full-row load an immediate offset
#pragma unroll
      for (int r = 0; r < BATCH; ++r)
        if (r0 + r < nfull) raw[r] = load_raw<DT>(p + ((r0 + r) & ~7) * STRIDE + ((r0 + r) & 7) * STRIDE);
#pragma unroll
      for (int r = 0; r < BATCH; ++r)
        if (r0 + r < nfull)
          process_match<DT, WMODE, BUILD, WRITE, false>(raw[r], true, m0 + (r0 + r) * STRIDE, E, fdelta, tau,
                                                        weights, w_out, r_out, acc, nkept);
    }
  }
  if (one_tail) {
    process_match<DT, WMODE, BUILD, WRITE, true>(traw, tok, tok ? start + ti : start, E, fdelta, tau, weights,
                                                 w_out, r_out, acc, nkept);
  } else {
    // several checked rows: only a wavefront whose four pair slots are not
    // all filled (at most one per row count) comes here
    for (int r = nfull; r < nrows; ++r) {
      const int i = r * STRIDE + lid;
      const bool ok = i < count;
      const RawT raw = load_raw<DT>(ok ? p + r * STRIDE : base);
      process_match<DT, WMODE, BUILD, WRITE, true>(raw, ok, ok ? start + i : start, E, fdelta, tau, weights, w_out,
                                                   r_out, acc, nkept);
    }
  }
}

// Reduce-scatter of 36 values over one 16-lane row (lane bits 3..0, DPP):
// each lane keeps 3 of the row's totals; value k of lane l is entry
// z + 5 b1 + 9 b2 + 18 b3 with z = k + 3 b0, valid if z < 5 and z + 5 b1 < 9.
__device__ inline void row_reduce_scatter36(const float (&a)[36], int lane, float (&out)[3]) {
  float b[18], c[9], d[5];
  rs_stage<36, 3>(a, b, lane);
  rs_stage<18, 2>(b, c, lane);
  rs_stage<9, 1>(c, d, lane);
  rs_stage<5, 0>(d, out, lane);
}

// The Gram pass (work items in dispatch order, longest first, so the
// wavefronts that wait for a free slot are the short ones).  Work item
// w < n_big: one wavefront on chunk big_chunk[w] (<= 64 big_rows(DT)
// matches: 1024, or 4096 for BF16; lanes strided so each load instruction
// reads one contiguous span) of a pair with more than small_max(DT) matches.
// Work item w >= n_big: one wavefront on four pairs of at most small_max(DT)
// matches, 16 lanes each (groups of pairs with equal row counts, built at
// set-up; a pair without matches stores zeros).  Each pair's sums are
// reduced over its lanes in a fixed order; a pair whose matches one
// wavefront covered stores its Gram directly (float64 of the float32 sum),
// the others leave chunk partials (slot big_slot[w]) for k_gram_finalize.
// An IRLS pass adds its wavefronts' kept-match counts into kept_slots.
template <int DT, int WMODE, bool BUILD, bool WRITE>
__global__ __launch_bounds__(kGramWaves * kLanes) void k_gram_pass(
    const void* __restrict__ uv, const int64_t* __restrict__ off, const int32_t* __restrict__ big_pair,
    const int32_t* __restrict__ big_chunk, const int32_t* __restrict__ big_slot,
    int64_t n_big, const int32_t* __restrict__ groups, int64_t n_groups, const float* __restrict__ weights, const double* __restrict__ ess, double delta, double tau,
    float* __restrict__ partials, double* __restrict__ W64, float* __restrict__ W32, float* __restrict__ w_out,
    float* __restrict__ r_out, unsigned long long* __restrict__ kept_slots) {
  // rows loaded per batch (measured on the medium scene, FP32: 1 row
  // 13.6-13.9 us, 2 rows 14.4-14.9, 4 rows 15.6, 8 rows 17.0; BF16 is bound
  // by vector ALU issue and loads 16 rows of a batch at once)
  constexpr int kBatch = (DT == FM_F64) ? 4 : (DT == FM_F32 ? 1 : kPerLane);
  const int lane = threadIdx.x & (kLanes - 1);
  // wave-uniform work item (scalar registers: the big path's pair data and
  // E_n are then scalar loads)
  const int64_t w = (int64_t)blockIdx.x * kGramWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t items = n_big + n_groups;
  if (w >= items) return;  // whole wavefront
  const float fdelta = (float)delta;
  float acc[36];
#pragma unroll
  for (int k = 0; k < 36; ++k) acc[k] = 0.0f;
  unsigned nkept = 0;
  double E[9];
  if (w < n_big) {
    const int64_t n = big_pair[w];
    const int32_t ps = big_slot[w];
    constexpr int kRows = big_rows(DT);
    constexpr int64_t kCh = (int64_t)kLanes * kRows;
    const int64_t start = off[n] + (int64_t)big_chunk[w] * kCh;
    const int count = (int)min(off[n + 1] - start, kCh);
    if constexpr (WMODE == W_IRLS) {
      // E_n is uniform here; held in vector registers all the same, since a
      // float64 FMA may read only one scalar operand
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        E[k] = ess[n * 9 + k];
        asm volatile("" : "+v"(E[k]));
      }
    }
    stream_rows<DT, WMODE, BUILD, WRITE, kLanes, kBatch, kRows>(uv, start, count, lane, (count + kLanes - 1) / kLanes,
                                                               count / kLanes, E, fdelta, tau, weights, w_out, r_out,
                                                               acc, nkept);
    if constexpr (BUILD) {
      int slot;
      const float v = wave_reduce_scatter36(acc, lane, slot);
      if (slot >= 0) {
        if (ps < 0) {
          if (W64) W64[n * 36 + slot] = (double)v;
          if (W32) W32[n * 36 + slot] = v;
        } else {
          partials[(int64_t)ps * 36 + slot] = v;
        }
      }
    }
  } else {
    constexpr int kGRows = group_rows(DT);
    const int l16 = lane & 15;
    const int64_t n = groups[(w - n_big) * 4 + (lane >> 4)];
    const bool have = n >= 0;
    const int64_t start = have ? off[n] : 0;
    const int count = have ? (int)(off[n + 1] - start) : 0;
    // the four pairs of a group have the same row count; rows before the
    // last are full unless a pair slot is unused; a group of pairs without
    // matches has no rows
    int nrows = (count + 15) >> 4;
    nrows = max(nrows, __shfl_xor(nrows, 16));
    nrows = max(nrows, __shfl_xor(nrows, 32));
    nrows = __builtin_amdgcn_readfirstlane(nrows);
    if (nrows > 0) {
      const int nfull = (__ballot(!have) == 0ull) ? nrows - 1 : 0;
      if constexpr (WMODE == W_IRLS) {
#pragma unroll
        for (int k = 0; k < 9; ++k) E[k] = have ? ess[n * 9 + k] : 0.0;
      }
      stream_rows<DT, WMODE, BUILD, WRITE, 16, kBatch, kGRows>(uv, start, count, l16, nrows, nfull, E, fdelta, tau,
                                                              weights, w_out, r_out, acc, nkept);
    }
    if constexpr (BUILD) {
      float v[3];
      row_reduce_scatter36(acc, lane, v);
      const int b0 = l16 & 1, b1 = (l16 >> 1) & 1, b2 = (l16 >> 2) & 1, b3 = (l16 >> 3) & 1;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int z = k + 3 * b0;
        if (have && z < 5 && z + 5 * b1 < 9) {
          const int slot = z + 5 * b1 + 9 * b2 + 18 * b3;
          if (W64) W64[n * 36 + slot] = (double)v[k];
          if (W32) W32[n * 36 + slot] = v[k];
        }
      }
    }
  }
  if constexpr (WMODE == W_IRLS) {
    // integer count (wave-uniform), spread over kKeptSlots counters (a
    // single address would serialise one atomic per wavefront); exact and
    // order-free
    if (lane == 0 && nkept) atomicAdd(&kept_slots[(w % kKeptSlots) * 16], (unsigned long long)nkept);
  }
}

// Total of the kept-match counters by one block of kKeptSlots threads; the
// counters are cleared for the next pass.
__device__ inline void sum_kept(unsigned long long* __restrict__ kept_slots, int64_t* __restrict__ kept) {
  __shared__ unsigned long long part[kKeptSlots / 64];
  unsigned long long s = 0;
  if (threadIdx.x < kKeptSlots) {
    s = kept_slots[threadIdx.x * 16];
    kept_slots[threadIdx.x * 16] = 0ull;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0 && threadIdx.x < kKeptSlots) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int k = 0; k < kKeptSlots / 64; ++k) t += part[k];
    *kept = (int64_t)t;
  }
}

// Gram of every pair that spans several work items: the sum of its chunk
// partials (chunks of `chunk` matches) in float64, in chunk order (the other
// pairs, empty ones included, were written by the pass itself).  Block 0
// also totals the kept counts of an IRLS pass (kept != NULL).
__global__ __launch_bounds__(kBlock) void k_gram_finalize(const float* __restrict__ partials,
                                                          const int64_t* __restrict__ off,
                                                          const int32_t* __restrict__ multi,
                                                          const int64_t* __restrict__ multi_first, int64_t n_multi,
                                                          int64_t chunk, double* __restrict__ W64,
                                                          float* __restrict__ W32,
                                                          unsigned long long* __restrict__ kept_slots,
                                                          int64_t* __restrict__ kept) {
  if (kept && blockIdx.x == 0) sum_kept(kept_slots, kept);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_multi * 36) return;
  const int64_t i = t / 36;
  const int64_t n = multi[i];
  const int k = (int)(t % 36);
  const int64_t chunks = (off[n + 1] - off[n] + chunk - 1) / chunk;
  double s = 0.0;
  for (int64_t j = 0; j < chunks; ++j) s += (double)partials[(multi_first[i] + j) * 36 + k];
  if (W64) W64[n * 36 + k] = s;
  if (W32) W32[n * 36 + k] = (float)s;
}

// Check mode: flags a non-finite coordinate among the stored matches.
template <int DT>
__global__ __launch_bounds__(kBlock) void k_check_coords(const void* __restrict__ uv, int64_t M,
                                                         unsigned* __restrict__ flag) {
  using RawT = typename RawMatch<DT>::T;
  bool bad = false;
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < M; m += (int64_t)gridDim.x * blockDim.x) {
    float4 f;
    double x[4];
    unpack<DT>(load_raw<DT>(reinterpret_cast<const RawT*>(uv) + m), f, x);
    bad = bad || !(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]) && isfinite(x[3]));
  }
  if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(flag, FM_CHECK_COORDS);
}

// E_n for every pair at the given poses (float64), for the residual pass.
// In check mode (flag != NULL) a pair whose |t_ij| is at most 1e-7 of
// |t_i| + |t_j| (below the resolution of float32 parameters, so its direction
// is rounding noise; exactly 0 included) or whose E_n is not finite (from
// non-finite parameters) is flagged.
__global__ void k_pair_essentials(const float* __restrict__ params, const int32_t* __restrict__ cams,
                                  int64_t P, double* __restrict__ ess, unsigned* __restrict__ flag) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= P) return;
  double a1[3], a2[3], ti[3], tj[3];
  double Ri[3][3], Rj[3][3], Rij[3][3], th[3], E[3][3];
  load_pose(params, cams[2 * n], a1, a2, ti);
  gs_matrix(gs_forward(a1, a2), Ri);
  load_pose(params, cams[2 * n + 1], a1, a2, tj);
  gs_matrix(gs_forward(a1, a2), Rj);
  const double ns = pair_essential(Ri, ti, Rj, tj, Rij, th, E);
  if (flag) {
    const double tn = sqrt(ti[0] * ti[0] + ti[1] * ti[1] + ti[2] * ti[2]) +
                      sqrt(tj[0] * tj[0] + tj[1] * tj[1] + tj[2] * tj[2]);
    unsigned bits = ns <= 1e-7 * tn ? FM_CHECK_DEGENERATE : 0u;
    bool fin = isfinite(ns);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) fin = fin && isfinite(E[a][b]);
    if (!fin) bits |= FM_CHECK_PARAMS;
    if (bits) atomicOr(flag, bits);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) ess[n * 9 + 3 * a + b] = E[a][b];
}

// ------------------------------------------------------------------ host side

template <int WMODE, bool BUILD, bool WRITE>
static fm_status launch_pass(fm_scene* s, const float* weights, double delta, double tau, double* W64,
                             float* W32, float* w_out, float* r_out, hipStream_t st) {
  const int64_t items = s->n_big + s->n_groups;
  if (items == 0) return FM_OK;
  const dim3 grid(grid_for(items, kGramWaves)), block(kGramWaves * kLanes);
  fm_timed timer(s->ctx, FM_K_GRAM, st, true);
#define FM_GRAM_ARGS                                                                                          \
  s->uv, s->offsets, s->big_pair, s->big_chunk, s->big_slot, s->n_big, s->groups, s->n_groups, weights, s->ess,   \
      delta, tau, s->partials, W64, W32, w_out, r_out, s->kept_slots
  switch (s->dtype) {
    case FM_F32:
      hipExtLaunchKernelGGL((k_gram_pass<FM_F32, WMODE, BUILD, WRITE>), grid, block, 0, st, timer.a, timer.b, 0,
                            FM_GRAM_ARGS);
      break;
    case FM_BF16:
      hipExtLaunchKernelGGL((k_gram_pass<FM_BF16, WMODE, BUILD, WRITE>), grid, block, 0, st, timer.a, timer.b, 0,
                            FM_GRAM_ARGS);
      break;
    default:
      hipExtLaunchKernelGGL((k_gram_pass<FM_F64, WMODE, BUILD, WRITE>), grid, block, 0, st, timer.a, timer.b, 0,
                            FM_GRAM_ARGS);
      break;
  }
#undef FM_GRAM_ARGS
  FM_CHECK_LAUNCH(s->ctx);
  return FM_OK;
}

// The multi-chunk sums and (with kept) the kept-match total; launched only
// when there is something to do.
static fm_status launch_finalize(fm_scene* s, double* W64, float* W32, int64_t* kept, hipStream_t st) {
  if (s->n_multi == 0 && !kept) return FM_OK;
  fm_timed timer(s->ctx, FM_K_FINALIZE, st, true);
  const int64_t nthreads = s->n_multi * 36 > 0 ? s->n_multi * 36 : 1;
  hipExtLaunchKernelGGL(k_gram_finalize, dim3(grid_for(nthreads, kBlock)), dim3(kBlock), 0, st, timer.a, timer.b, 0,
                        s->partials, s->offsets, s->multi, s->multi_first, s->n_multi, s->chunk, W64, W32,
                        s->kept_slots, kept);
  FM_CHECK_LAUNCH(s->ctx);
  return FM_OK;
}

static fm_status launch_essentials(fm_scene* s, const float* params, hipStream_t st) {
  fm_timed timer(s->ctx, FM_K_ESSENTIALS, st, true);
  hipExtLaunchKernelGGL(k_pair_essentials, dim3(grid_for(s->P > 0 ? s->P : 1, kBlock)), dim3(kBlock), 0, st, timer.a,
                        timer.b, 0, params, (const int32_t*)s->pair_cams, s->P, s->ess,
                        s->ctx->check ? s->ctx->check_flag : nullptr);
  FM_CHECK_LAUNCH(s->ctx);
  return FM_OK;
}

fm_status fm_launch_essentials(fm_scene* s, const float* params, hipStream_t st) {
  return launch_essentials(s, params, st);
}

// Check mode: one extra pass over the stored coordinates.
static fm_status launch_check_coords(fm_scene* s, hipStream_t st) {
  if (!s->ctx->check || s->M == 0) return FM_OK;
  const int64_t want = grid_for(s->M, kBlock);
  const dim3 grid((unsigned)(want < 4096 ? want : 4096)), block(kBlock);
  switch (s->dtype) {
    case FM_F32:
      hipLaunchKernelGGL(k_check_coords<FM_F32>, grid, block, 0, st, s->uv, s->M, s->ctx->check_flag);
      break;
    case FM_BF16:
      hipLaunchKernelGGL(k_check_coords<FM_BF16>, grid, block, 0, st, s->uv, s->M, s->ctx->check_flag);
      break;
    default:
      hipLaunchKernelGGL(k_check_coords<FM_F64>, grid, block, 0, st, s->uv, s->M, s->ctx->check_flag);
      break;
  }
  FM_CHECK_LAUNCH(s->ctx);
  return FM_OK;
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
  if ((rc = launch_check_coords(s, st)) != FM_OK) return rc;
  fm_timed call(ctx, FM_K_GRAM_CALL, st);
  rc = weights ? launch_pass<W_ARRAY, true, false>(s, weights, 0, 0, W64, W32, nullptr, nullptr, st)
               : launch_pass<W_UNIT, true, false>(s, nullptr, 0, 0, W64, W32, nullptr, nullptr, st);
  if (rc != FM_OK) return rc;
  return launch_finalize(s, W64, W32, nullptr, st);
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
  if ((rc = launch_check_coords(s, st)) != FM_OK) return rc;
  fm_timed call(ctx, FM_K_GRAM_CALL, st);
  if ((rc = launch_essentials(s, params, st)) != FM_OK) return rc;
  if ((rc = launch_pass<W_IRLS, false, true>(s, nullptr, delta, tau, nullptr, nullptr, w_out, r_out, st)) != FM_OK)
    return rc;
  return launch_finalize(s, nullptr, nullptr, kept, st);
}

extern "C" fm_status fm_reweight_build(fm_ctx* ctx, fm_scene* s, const float* params, float delta, float tau,
                                       double* W64, float* W32, int64_t* kept, fm_stream stream) {
  fm_status rc = check_scene(ctx, s, "fm_reweight_build");
  if (rc != FM_OK) return rc;
  if ((rc = check_irls_args(ctx, "fm_reweight_build", params, delta, tau, kept)) != FM_OK) return rc;
  if (!W64 && !W32 && s->P > 0) return fm_fail(ctx, FM_EINVAL, "fm_reweight_build: both outputs are NULL");
  hipStream_t st = (hipStream_t)stream;
  if ((rc = launch_check_coords(s, st)) != FM_OK) return rc;
  fm_timed call(ctx, FM_K_GRAM_CALL, st);
  if ((rc = launch_essentials(s, params, st)) != FM_OK) return rc;
  if ((rc = launch_pass<W_IRLS, true, false>(s, nullptr, delta, tau, W64, W32, nullptr, nullptr, st)) != FM_OK)
    return rc;
  return launch_finalize(s, W64, W32, kept, st);
}
