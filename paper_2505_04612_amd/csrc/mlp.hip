// Learned per-match weights: feature extraction and a 3 -> 64 -> 64 -> 1 MLP
// (ReLU, ReLU, sigmoid) whose 64x64 layer runs on MFMA (float16 operands,
// float32 accumulation), forward and backward.
//
// MFMA layouts (one wavefront, lane l, r = l % 16, q = l / 16), both with
// the 16x16 float32 result D[4q + j][r] in four registers:
//   v_mfma_f32_16x16x32_f16 (gfx950): operand A (16 x 32, M x K) holds
//     A[r][8q + j] in its 8 halves, operand B (32 x 16) holds B[8q + j][r];
//     used where the contraction runs over the 64 hidden units (the
//     forward's 64x64 layer, the backward's dh1 = dh2 W2): two per 16x16
//     output tile;
//   v_mfma_f32_16x16x16_f16: A[r][4q + j], B[4q + j][r]; used for the
//     backward's dW2, whose contraction runs over a 16-match tile, and for
//     the forward's 64 -> 1 layer, whose operand B is the transposed 64x64
//     layer's result as it stands (units along 4q + j, matches along r).
// A tile is 16 matches; lanes r = 0..15 of each quarter q address one match
// (operand A) or one output unit (result).
#include <mutex>

#include "fm_internal.h"

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kHid = 64;
// gradient entries: W2 (64x64), b2, W3, b3, W1 (64x3), b1
constexpr int kG_W2 = 0, kG_b2 = 4096, kG_W3 = 4160, kG_b3 = 4224, kG_W1 = 4225, kG_b1 = 4417, kG_N = 4481;

struct MlpPtrs {
  const float *W1, *b1, *W2, *b2, *W3, *b3, *mean, *std;
};

__device__ inline f4 mfma16(h4 a, h4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0); }
__device__ inline f4 mfma32(h8 a, h8 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }

constexpr float kLog2e = 1.4426950408889634f;

struct MlpLds {
  float W1[kHid * 3], b1[kHid], b2[kHid], W3[kHid], mean[3], rstd[3], b3;
};

__device__ inline void load_lds(const MlpPtrs& w, MlpLds& s) {
  for (int k = threadIdx.x; k < kHid * 3; k += blockDim.x) s.W1[k] = w.W1[k];
  for (int k = threadIdx.x; k < kHid; k += blockDim.x) {
    s.b1[k] = w.b1[k];
    s.b2[k] = w.b2[k];
    s.W3[k] = w.W3[k];
  }
  if (threadIdx.x < 3) {
    s.mean[threadIdx.x] = w.mean[threadIdx.x];
    s.rstd[threadIdx.x] = 1.0f / w.std[threadIdx.x];
  }
  if (threadIdx.x == 0) s.b3 = w.b3[0];
  __syncthreads();
}

__device__ inline void load_x(const float* feats, int64_t m, const MlpLds& s, float x[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) x[c] = (feats[m * 3 + c] - s.mean[c]) * s.rstd[c];
}

// Blocks of 4 wavefronts walk the 16-match tiles in block-uniform steps (so
// block barriers are safe); tile = step * 4 * gridDim + 4 * block + wave.
// KEEP: also store each match's 128 FP16 activations to act (what the
// backward reads back); the plain forward is instantiated without that code.
template <bool KEEP>
__global__ __launch_bounds__(256, 4) void k_mlp_forward(int64_t M, const float* __restrict__ feats, MlpPtrs w,
                                                     float out_scale, float* __restrict__ out,
                                                     _Float16* __restrict__ act) {
  __shared__ MlpLds s;
  // per-wavefront staging of the kept activations: rows padded by 16 bytes,
  // so that the 16 rows a store instruction touches start in different banks
  constexpr int kTstRow = 2 * kHid + 8;
  __shared__ __attribute__((aligned(16))) _Float16 Tst[4][16][kTstRow];
  load_lds(w, s);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  // layer-2 operand B[k][n] = W2[n][k] for k-tile kk (32 inputs), n-tile nt
  h8 B[2][4];
#pragma unroll
  for (int kk = 0; kk < 2; ++kk)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int j = 0; j < 8; ++j) B[kk][nt][j] = (_Float16)w.W2[(16 * nt + r) * kHid + 32 * kk + 8 * q + j];
  // output-layer operand A3[n][k] for units k of n-tile nt: row 0 holds W3
  // (as float16 high and low parts, so the products keep float32
  // precision), rows 1..15 are zero; lane (q, r) holds A3[r][4q + j]
  h4 W3h[4], W3l[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float w3 = r == 0 ? w.W3[16 * nt + 4 * q + j] : 0.0f;
      W3h[nt][j] = (_Float16)w3;
      W3l[nt][j] = (_Float16)(w3 - (float)W3h[nt][j]);
    }
  const int64_t ntiles = (M + 15) / 16;
  for (int64_t base = (int64_t)blockIdx.x * 4; base < ntiles; base += (int64_t)gridDim.x * 4) {
    const int64_t tile = base + wave;
    if (tile >= ntiles) continue;   // no block barrier below
    const int64_t m = tile * 16 + r;
    const bool ok = m < M;
    float x[3];
    load_x(feats, ok ? m : M - 1, s, x);
    h8 A[2];
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = 32 * kk + 8 * q + j;
        const float z = fmaf(s.W1[3 * k], x[0], fmaf(s.W1[3 * k + 1], x[1], fmaf(s.W1[3 * k + 2], x[2], s.b1[k])));
        A[kk][j] = (_Float16)fmaxf(z, 0.0f);
      }
    // layer 2 transposed (W2 as operand A, the tile's layer-1 activations as
    // operand B): C[nt][j] = z2 of unit 16 nt + 4q + j, match 16 tile + r,
    // which after bias, ReLU and rounding to float16 is operand B of the
    // output layer's 16x16x16 MFMA as it stands (units along 4q + j)
    f4 Z = f4{0.0f, 0.0f, 0.0f, 0.0f};
    h4 h[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f4 C = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) C = mfma32(B[kk][nt], A[kk], C);
#pragma unroll
      for (int j = 0; j < 4; ++j) h[nt][j] = (_Float16)fmaxf(C[j] + s.b2[16 * nt + 4 * q + j], 0.0f);
      Z = mfma16(W3h[nt], h[nt], Z);
      Z = mfma16(W3l[nt], h[nt], Z);
    }
    // the tile's activations (16 rows of 128 halves: one contiguous 4 KB
    // block of act) through this wavefront's LDS rows, then written with
    // consecutive 16-byte stores; LDS operations of a wavefront complete in
    // order, the fences keep the compiler from reordering them
    if constexpr (KEEP) {
      _Float16* T = &Tst[wave][0][0];
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) *reinterpret_cast<h8*>(T + r * kTstRow + 32 * kk + 8 * q) = A[kk];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) *reinterpret_cast<h4*>(T + r * kTstRow + 64 + 16 * nt + 4 * q) = h[nt];
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = lane + 64 * i, row = c >> 4, col = 8 * (c & 15);
        const int64_t mr = tile * 16 + row;
        if (mr < M) *reinterpret_cast<h8*>(act + mr * 128 + col) = *reinterpret_cast<const h8*>(T + row * kTstRow + col);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    // Z[j] = row 4q + j of A3 H2^T: row 0 (lanes q = 0, register 0) is z3 of
    // match 16 tile + r; the sigmoid on the hardware 2^x and reciprocal
    // (~1 ulp each)
    const float e = __builtin_amdgcn_exp2f(-(Z[0] + s.b3) * kLog2e);
    if (q == 0 && ok) out[m] = out_scale * __builtin_amdgcn_rcpf(1.0f + e);
  }
}

// Backward of sum_m dout[m] * sigmoid(z3[m]) from the stored activations.
// Each wavefront accumulates its gradient contributions in registers and
// writes them to its own slot of `part` [waves, kG_N]; k_mlp_reduce adds the
// slots in a fixed order.
__global__ __launch_bounds__(256) void k_mlp_backward(int64_t M, const float* __restrict__ feats, MlpPtrs w,
                                                      const _Float16* __restrict__ act,
                                                      const float* __restrict__ dout, float* __restrict__ part) {
  __shared__ MlpLds s;
  __shared__ _Float16 T[4][16][kHid + 4];   // per-wave transpose of dh2
  // per-wave copy of the tile's activations (16 matches x 128, rows padded
  // so that the four row groups a read instruction touches use different
  // banks): read from global memory in 16-byte pieces, then per unit
  __shared__ _Float16 Ast[4][16][2 * kHid + 8];
  load_lds(w, s);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  // operand B of dh1 = dh2 W2: B[k = o][n = i] = W2[o][i], k-tiles of 32
  h8 B2[2][4];
#pragma unroll
  for (int kt = 0; kt < 2; ++kt)
#pragma unroll
    for (int it = 0; it < 4; ++it)
#pragma unroll
      for (int j = 0; j < 8; ++j) B2[kt][it][j] = (_Float16)w.W2[(32 * kt + 8 * q + j) * kHid + 16 * it + r];
  f4 gW2[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) gW2[a][b] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  float gW3[4] = {0, 0, 0, 0}, gb2[4] = {0, 0, 0, 0}, gb1[4] = {0, 0, 0, 0}, gb3 = 0.0f;
  float gW1[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  const int64_t ntiles = (M + 15) / 16;
  for (int64_t base = (int64_t)blockIdx.x * 4; base < ntiles; base += (int64_t)gridDim.x * 4) {
    const int64_t tile = base + wave;
    const bool tv = tile < ntiles;
    // the tile's 16 x 128 activations (4 KB, 256 pieces of 16 bytes; rows
    // past M are zeros)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int idx = 64 * t + lane, row = idx >> 4, piece = idx & 15;
      const int64_t m = tile * 16 + row;
      h8 v;
      if (tv && m < M) {
        v = *reinterpret_cast<const h8*>(act + m * 128 + 8 * piece);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (_Float16)0.0f;
      }
      *reinterpret_cast<h8*>(&Ast[wave][row][8 * piece]) = v;
    }
    __syncthreads();
    // this lane's result-layout rows 4q + j
    float h2[4][4], h1[4][4], d3[4], x[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t row = tile * 16 + 4 * q + j;
      const bool ok = tv && row < M;
      const int64_t rc = ok ? row : 0;
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        h2[j][nt] = (float)Ast[wave][4 * q + j][64 + 16 * nt + r];
        h1[j][nt] = (float)Ast[wave][4 * q + j][16 * nt + r];
      }
      float z = 0.0f;
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) z = fmaf(s.W3[16 * nt + r], h2[j][nt], z);
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) z += __shfl_xor(z, o);
      const float sg = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-(z + s.b3) * kLog2e));
      d3[j] = ok ? dout[rc] * sg * (1.0f - sg) : 0.0f;
      if (ok) load_x(feats, rc, s, x[j]);
      else x[j][0] = x[j][1] = x[j][2] = 0.0f;
    }
    // dh2 (result layout), dW3, db2, db3
    h4 A2[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float dh = h2[j][nt] > 0.0f ? d3[j] * s.W3[16 * nt + r] : 0.0f;
        gW3[nt] = fmaf(d3[j], h2[j][nt], gW3[nt]);
        gb2[nt] += dh;
        A2[nt][j] = (_Float16)dh;
        T[wave][4 * q + j][16 * nt + r] = (_Float16)dh;
      }
    if (r == 0) gb3 += d3[0] + d3[1] + d3[2] + d3[3];
    // dW2[o][i] += sum_m dh2[m][o] h1[m][i]
    h4 B1[4];
#pragma unroll
    for (int it = 0; it < 4; ++it)
#pragma unroll
      for (int j = 0; j < 4; ++j) B1[it][j] = (_Float16)h1[j][it];
#pragma unroll
    for (int ot = 0; ot < 4; ++ot)
#pragma unroll
      for (int it = 0; it < 4; ++it) gW2[ot][it] = mfma16(A2[ot], B1[it], gW2[ot][it]);
    __syncthreads();
    // dh1 = (dh2 W2) * (h1 > 0): operand A[m][o] read back transposed
    h8 A3[2];
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
      for (int j = 0; j < 8; ++j) A3[kt][j] = T[wave][r][32 * kt + 8 * q + j];
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      f4 C = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kt = 0; kt < 2; ++kt) C = mfma32(A3[kt], B2[kt][it], C);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float dh1 = h1[j][it] > 0.0f ? C[j] : 0.0f;
        gb1[it] += dh1;
#pragma unroll
        for (int c = 0; c < 3; ++c) gW1[it][c] = fmaf(dh1, x[j][c], gW1[it][c]);
      }
    }
    __syncthreads();
  }
  // write this wavefront's slot
  const int64_t slot = (int64_t)blockIdx.x * 4 + wave;
  float* P = part + slot * kG_N;
#pragma unroll
  for (int ot = 0; ot < 4; ++ot)
#pragma unroll
    for (int it = 0; it < 4; ++it)
#pragma unroll
      for (int j = 0; j < 4; ++j) P[kG_W2 + (16 * ot + 4 * q + j) * kHid + 16 * it + r] = gW2[ot][it][j];
  // per-unit sums: add the four quarters (lanes r, r+16, r+32, r+48)
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    for (int o = 16; o < 64; o <<= 1) {
      gW3[nt] += __shfl_xor(gW3[nt], o);
      gb2[nt] += __shfl_xor(gb2[nt], o);
      gb1[nt] += __shfl_xor(gb1[nt], o);
#pragma unroll
      for (int c = 0; c < 3; ++c) gW1[nt][c] += __shfl_xor(gW1[nt][c], o);
    }
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) gb3 += __shfl_xor(gb3, o);
  if (q == 0) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int u = 16 * nt + r;
      P[kG_W3 + u] = gW3[nt];
      P[kG_b2 + u] = gb2[nt];
      P[kG_b1 + u] = gb1[nt];
#pragma unroll
      for (int c = 0; c < 3; ++c) P[kG_W1 + 3 * u + c] = gW1[nt][c];
    }
  }
  if (lane == 0) P[kG_b3] = gb3;
}

struct MlpGradPtrs {
  float *W1, *b1, *W2, *b2, *W3, *b3;
};

// Sum of the gradient slots, entry by entry: each workgroup takes 64
// entries (one per lane, coalesced over the slots' rows); its kRedWaves
// wavefronts take consecutive ranges of the slots, eight running sums per
// lane so that eight loads are in flight, and the wavefronts' sums are added
// in wavefront order: a fixed order for any slot count.
constexpr int kRedWaves = 16;

__global__ __launch_bounds__(64 * kRedWaves) void k_mlp_reduce(const float* __restrict__ part, int64_t slots,
                                                              MlpGradPtrs g) {
  __shared__ float red[kRedWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  const int64_t per = (slots + kRedWaves - 1) / kRedWaves;
  const int64_t k0 = wave * per, k1 = min(slots, k0 + per);
  float p[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  if (e < kG_N) {
    int64_t k = k0;
    for (; k + 8 <= k1; k += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) p[u] += part[(k + u) * kG_N + e];
    }
    for (; k < k1; ++k) p[0] += part[k * kG_N + e];
  }
  red[wave][lane] = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
  __syncthreads();
  if (wave != 0 || e >= kG_N) return;
  float s = 0.0f;
#pragma unroll
  for (int w = 0; w < kRedWaves; ++w) s += red[w][lane];
  if (e < kG_b2) g.W2[e] = s;
  else if (e < kG_W3) g.b2[e - kG_b2] = s;
  else if (e < kG_b3) g.W3[e - kG_W3] = s;
  else if (e < kG_W1) g.b3[0] = s;
  else if (e < kG_b1) g.W1[e - kG_W1] = s;
  else g.b1[e - kG_b1] = s;
}

// ------------------------------------------------------------------ features

// Per match: f0 = log max(|r|, delta) with r = x2~^T E_n x1~ (float64),
// f1 = log |Q_n|, f2 = angle between R_i^T x1~ and R_j^T x2~.  One wavefront
// per Gram work item; E_n comes from the per-pair essentials pass.
template <int DT>
__global__ __launch_bounds__(256) void k_features(const void* __restrict__ uv, const int64_t* __restrict__ off,
                                                  const int64_t* __restrict__ wi_off, int64_t P, int64_t n_wi,
                                                  const int32_t* __restrict__ cams, const float* __restrict__ params,
                                                  const double* __restrict__ ess, double delta,
                                                  float* __restrict__ feats) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= n_wi) return;
  int64_t lo = 0, hi = P;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (wi_off[mid] <= w) lo = mid; else hi = mid;
  }
  const int64_t n = lo;
  const int64_t start = off[n] + (w - wi_off[n]) * kChunk;
  const int64_t stop = min(off[n + 1], start + kChunk);
  const float f1 = logf((float)(off[n + 1] - off[n]));
  double E[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) E[k] = ess[n * 9 + k];
  double a1[3], a2[3], t[3], Ri[3][3], Rj[3][3];
  load_pose(params, cams[2 * n], a1, a2, t);
  gs_matrix(gs_forward(a1, a2), Ri);
  load_pose(params, cams[2 * n + 1], a1, a2, t);
  gs_matrix(gs_forward(a1, a2), Rj);
  for (int64_t m = start + lane; m < stop; m += kLanes) {
    double x[4];
    if constexpr (DT == FM_F32) {
      const float4 v = reinterpret_cast<const float4*>(uv)[m];
      x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    } else if constexpr (DT == FM_BF16) {
      const uint2 v = reinterpret_cast<const uint2*>(uv)[m];
      x[0] = __uint_as_float(v.x << 16); x[1] = __uint_as_float(v.x & 0xffff0000u);
      x[2] = __uint_as_float(v.y << 16); x[3] = __uint_as_float(v.y & 0xffff0000u);
    } else {
      const double2* d = reinterpret_cast<const double2*>(uv) + 2 * m;
      x[0] = d[0].x; x[1] = d[0].y; x[2] = d[1].x; x[3] = d[1].y;
    }
    const double e0 = E[0] * x[0] + E[1] * x[1] + E[2];
    const double e1 = E[3] * x[0] + E[4] * x[1] + E[5];
    const double e2 = E[6] * x[0] + E[7] * x[1] + E[8];
    const double res = fabs(x[2] * e0 + x[3] * e1 + e2);
    double ra[3], rb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ra[c] = Ri[0][c] * x[0] + Ri[1][c] * x[1] + Ri[2][c];
      rb[c] = Rj[0][c] * x[2] + Rj[1][c] * x[3] + Rj[2][c];
    }
    const double cx = ra[1] * rb[2] - ra[2] * rb[1], cy = ra[2] * rb[0] - ra[0] * rb[2],
                 cz = ra[0] * rb[1] - ra[1] * rb[0];
    const double dotp = ra[0] * rb[0] + ra[1] * rb[1] + ra[2] * rb[2];
    feats[m * 3 + 0] = (float)log(res > delta ? res : delta);
    feats[m * 3 + 1] = f1;
    feats[m * 3 + 2] = (float)atan2(sqrt(cx * cx + cy * cy + cz * cz), dotp);
  }
}

// ------------------------------------------------------------------ host side

static fm_status mlp_ptrs(fm_ctx* ctx, const fm_mlp* w, MlpPtrs& p) {
  if (!w || !w->W1 || !w->b1 || !w->W2 || !w->b2 || !w->W3 || !w->b3 || !w->feat_mean || !w->feat_std)
    return fm_fail(ctx, FM_EINVAL, "MLP weight pointer is NULL");
  p = MlpPtrs{w->W1, w->b1, w->W2, w->b2, w->W3, w->b3, w->feat_mean, w->feat_std};
  return FM_OK;
}

static unsigned mlp_blocks(fm_ctx* ctx, int64_t M, int per_cu = 2) {
  const int64_t tiles = (M + 15) / 16;
  int64_t b = (tiles + 3) / 4;
  const int64_t cap = (int64_t)ctx->num_cu * per_cu;
  return (unsigned)(b < cap ? (b > 0 ? b : 1) : cap);
}

extern "C" fm_status fm_mlp_forward(fm_ctx* ctx, int64_t M, const float* feats, const fm_mlp* w, float out_scale,
                                    float* out, void* act, fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  if (M < 0) return fm_fail(ctx, FM_ESHAPE, "fm_mlp_forward: M < 0");
  MlpPtrs p;
  fm_status rc = mlp_ptrs(ctx, w, p);
  if (rc != FM_OK) return rc;
  if (M == 0) return FM_OK;
  if (!feats || !out) return fm_fail(ctx, FM_EINVAL, "fm_mlp_forward: NULL feats or out");
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  // four workgroups of four wavefronts per CU: the forward kernel's register
  // use allows four wavefronts per SIMD, and its per-tile chain (feature load,
  // layer 1 from LDS, MFMA, epilogue) needs them to hide its latency
  if (act)
    hipLaunchKernelGGL(k_mlp_forward<true>, dim3(mlp_blocks(ctx, M, 4)), dim3(256), 0, (hipStream_t)stream, M, feats,
                       p, out_scale, out, (_Float16*)act);
  else
    hipLaunchKernelGGL(k_mlp_forward<false>, dim3(mlp_blocks(ctx, M, 4)), dim3(256), 0, (hipStream_t)stream, M, feats,
                       p, out_scale, out, (_Float16*)nullptr);
  FM_CHECK_LAUNCH(ctx);
  return FM_OK;
}

extern "C" fm_status fm_mlp_backward(fm_ctx* ctx, int64_t M, const float* feats, const fm_mlp* w, const void* act,
                                     const float* dout, fm_mlp_grad* g, fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  if (M < 0) return fm_fail(ctx, FM_ESHAPE, "fm_mlp_backward: M < 0");
  MlpPtrs p;
  fm_status rc = mlp_ptrs(ctx, w, p);
  if (rc != FM_OK) return rc;
  if (!g || !g->W1 || !g->b1 || !g->W2 || !g->b2 || !g->W3 || !g->b3)
    return fm_fail(ctx, FM_EINVAL, "fm_mlp_backward: gradient pointer is NULL");
  if (M > 0 && (!feats || !act || !dout)) return fm_fail(ctx, FM_EINVAL, "fm_mlp_backward: NULL input");
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  const unsigned blocks = mlp_blocks(ctx, M);
  const int64_t slots = (int64_t)blocks * 4;
  const size_t need = sizeof(float) * (size_t)slots * kG_N;
  if (ctx->ws_bytes < need) {
    FM_HIP_TRY(ctx, hipStreamSynchronize((hipStream_t)stream));
    (void)hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    hipError_t e = hipMalloc(&ctx->ws, need);
    if (e != hipSuccess) return fm_fail(ctx, FM_ENOMEM, "fm_mlp_backward: workspace: %s", hipGetErrorString(e));
    ctx->ws_bytes = need;
  }
  float* part = (float*)ctx->ws;
  if (M > 0) {
    hipLaunchKernelGGL(k_mlp_backward, dim3(blocks), dim3(256), 0, (hipStream_t)stream, M, feats, p,
                       (const _Float16*)act, dout, part);
    FM_CHECK_LAUNCH(ctx);
  }
  MlpGradPtrs gp{g->W1, g->b1, g->W2, g->b2, g->W3, g->b3};
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kG_N + 63) / 64), dim3(64 * kRedWaves), 0, (hipStream_t)stream, part,
                     M > 0 ? slots : (int64_t)0, gp);
  FM_CHECK_LAUNCH(ctx);
  return FM_OK;
}


extern "C" fm_status fm_match_features(fm_ctx* ctx, fm_scene* s, const float* params, float delta, float* feats,
                                       fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  if (!s || s->ctx != ctx) return fm_fail(ctx, FM_EINVAL, "fm_match_features: bad scene");
  if (!params || (!feats && s->M > 0)) return fm_fail(ctx, FM_EINVAL, "fm_match_features: NULL argument");
  if (!(delta > 0.0f)) return fm_fail(ctx, FM_EINVAL, "fm_match_features: delta must be > 0");
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  fm_status rc = fm_launch_essentials(s, params, st);
  if (rc != FM_OK || s->n_wi == 0) return rc;
  const dim3 grid(grid_for(s->n_wi, 4)), block(256);
  switch (s->dtype) {
    case FM_F32:
      hipLaunchKernelGGL(k_features<FM_F32>, grid, block, 0, st, s->uv, s->offsets, s->wi_off, s->P, s->n_wi,
                         s->pair_cams, params, s->ess, (double)delta, feats);
      break;
    case FM_BF16:
      hipLaunchKernelGGL(k_features<FM_BF16>, grid, block, 0, st, s->uv, s->offsets, s->wi_off, s->P, s->n_wi,
                         s->pair_cams, params, s->ess, (double)delta, feats);
      break;
    default:
      hipLaunchKernelGGL(k_features<FM_F64>, grid, block, 0, st, s->uv, s->offsets, s->wi_off, s->P, s->n_wi,
                         s->pair_cams, params, s->ess, (double)delta, feats);
      break;
  }
  FM_CHECK_LAUNCH(ctx);
  return FM_OK;
}

// ------------------------------------------------------------------ allocation-free backward

// Gradient slots of fm_mlp_backward_noalloc: a file-scope device array (each
// GPU the library runs on holds its own copy until the process ends) sized
// for kNoAllocBlocks workgroups of four wavefronts, 512 slots of kG_N floats
// (9.2 MB).  Host code never passes `scratch` itself to a kernel (its host
// name is a stand-in, not a device address): the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr int kNoAllocBlocks = 128;
constexpr int64_t kNoAllocSlots = (int64_t)kNoAllocBlocks * 4;
static __device__ __align__(256) float scratch[kNoAllocSlots * kG_N];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static float* g_scratch_dev[kMaxDevices];

// The device address of `scratch` on the context's device (which the caller
// has made current), looked up on the first call on that device.
static fm_status scratch_ptr(fm_ctx* ctx, float** out) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return fm_fail(ctx, FM_EINVAL, "fm_mlp_backward_noalloc: device %d beyond %d", ctx->device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[ctx->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fm_fail(ctx, FM_EHIP, "fm_mlp_backward_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
    g_scratch_dev[ctx->device] = (float*)p;
  }
  *out = g_scratch_dev[ctx->device];
  return FM_OK;
}

extern "C" fm_status fm_mlp_backward_noalloc(fm_ctx* ctx, int64_t M, const float* feats, const fm_mlp* w,
                                             const void* act, const float* dout, fm_mlp_grad* g, fm_stream stream) {
  if (!ctx) return FM_EINVAL;
  if (M < 0) return fm_fail(ctx, FM_ESHAPE, "fm_mlp_backward_noalloc: M < 0");
  MlpPtrs p;
  fm_status rc = mlp_ptrs(ctx, w, p);
  if (rc != FM_OK) return rc;
  if (!g || !g->W1 || !g->b1 || !g->W2 || !g->b2 || !g->W3 || !g->b3)
    return fm_fail(ctx, FM_EINVAL, "fm_mlp_backward_noalloc: gradient pointer is NULL");
  if (M > 0 && (!feats || !act || !dout)) return fm_fail(ctx, FM_EINVAL, "fm_mlp_backward_noalloc: NULL input");
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  float* part = nullptr;
  if ((rc = scratch_ptr(ctx, &part)) != FM_OK) return rc;
  // the launch of fm_mlp_backward, capped at the workgroups the scratch holds
  // slots for (identical launch, so identical results, up to 8,192 matches)
  unsigned blocks = mlp_blocks(ctx, M);
  if (blocks > (unsigned)kNoAllocBlocks) blocks = kNoAllocBlocks;
  const int64_t slots = (int64_t)blocks * 4;
  if (slots > kNoAllocSlots)
    return fm_fail(ctx, FM_ESHAPE, "fm_mlp_backward_noalloc: %lld gradient slots exceed the %lld the scratch holds",
                   (long long)slots, (long long)kNoAllocSlots);
  if (M > 0) {
    hipLaunchKernelGGL(k_mlp_backward, dim3(blocks), dim3(256), 0, (hipStream_t)stream, M, feats, p,
                       (const _Float16*)act, dout, part);
    FM_CHECK_LAUNCH(ctx);
  }
  MlpGradPtrs gp{g->W1, g->b1, g->W2, g->b2, g->W3, g->b3};
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kG_N + 63) / 64), dim3(64 * kRedWaves), 0, (hipStream_t)stream, part,
                     M > 0 ? slots : (int64_t)0, gp);
  FM_CHECK_LAUNCH(ctx);
  return FM_OK;
}
