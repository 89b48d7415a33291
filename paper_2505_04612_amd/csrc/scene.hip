// Context, error handling and scene set-up: validation of the pair/match
// structure, the Gram work-item table and the per-camera incidence lists.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <vector>

#include "fm_internal.h"
#include "gram_plan.h"

fm_status fm_fail(fm_ctx* ctx, fm_status st, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

extern "C" const char* fm_version(void) { return "fastmap_hip 0.1 gfx950"; }

extern "C" fm_status fm_create(fm_ctx** out, int device) {
  if (!out) return FM_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return FM_EINVAL;
  fm_ctx* ctx = new (std::nothrow) fm_ctx();
  if (!ctx) return FM_ENOMEM;
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess ||
      hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
    delete ctx;
    return FM_EHIP;
  }
  *out = ctx;
  return FM_OK;
}

static hipEvent_t pool_get(fm_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

fm_timed::fm_timed(fm_ctx* c, int k, hipStream_t s, bool dispatch) : ctx(c), kernel(k), st(s), at_dispatch(dispatch) {
  if (ctx && ctx->profile) {
    a = pool_get(ctx);
    b = pool_get(ctx);
    if (a && b && !at_dispatch) (void)hipEventRecord(a, st);
  }
}

fm_timed::~fm_timed() {
  if (a && b) {
    if (!at_dispatch) (void)hipEventRecord(b, st);
    ctx->timings.push_back({kernel, a, b});
  } else {
    if (a) ctx->event_pool.push_back(a);
    if (b) ctx->event_pool.push_back(b);
  }
}

static void release_timings(fm_ctx* ctx) {
  for (auto& t : ctx->timings) {
    ctx->event_pool.push_back(t.start);
    ctx->event_pool.push_back(t.stop);
  }
  ctx->timings.clear();
}

extern "C" fm_status fm_profile_enable(fm_ctx* ctx, int enable) {
  if (!ctx) return FM_EINVAL;
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  FM_HIP_TRY(ctx, hipDeviceSynchronize());
  release_timings(ctx);
  ctx->profile = enable != 0;
  return FM_OK;
}

extern "C" fm_status fm_profile_read(fm_ctx* ctx, int kernel, double* total_ms, int64_t* launches) {
  if (!ctx) return FM_EINVAL;
  if (!total_ms || !launches) return fm_fail(ctx, FM_EINVAL, "fm_profile_read: NULL output");
  if (kernel < 0 || kernel >= FM_K_COUNT) return fm_fail(ctx, FM_EINVAL, "fm_profile_read: unknown kernel %d", kernel);
  double sum = 0.0;
  int64_t n = 0;
  for (auto& t : ctx->timings) {
    if (t.kernel != kernel) continue;
    FM_HIP_TRY(ctx, hipEventSynchronize(t.stop));
    float ms = 0.0f;
    FM_HIP_TRY(ctx, hipEventElapsedTime(&ms, t.start, t.stop));
    sum += ms;
    ++n;
  }
  *total_ms = sum;
  *launches = n;
  return FM_OK;
}

extern "C" void fm_destroy(fm_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  release_timings(ctx);
  for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
  (void)hipFree(ctx->ws);
  (void)hipFree(ctx->check_flag);
  delete ctx;
}

// ------------------------------------------------------------------ check mode

extern "C" fm_status fm_set_check(fm_ctx* ctx, int enable) {
  if (!ctx) return FM_EINVAL;
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (enable && !ctx->check_flag) {
    FM_HIP_TRY(ctx, hipMalloc(&ctx->check_flag, sizeof(unsigned)));
    FM_HIP_TRY(ctx, hipMemset(ctx->check_flag, 0, sizeof(unsigned)));
    FM_HIP_TRY(ctx, hipDeviceSynchronize());
  }
  ctx->check = enable != 0;
  return FM_OK;
}

extern "C" fm_status fm_check(fm_ctx* ctx, fm_stream stream, uint32_t* flags) {
  if (!ctx) return FM_EINVAL;
  if (flags) *flags = 0;
  if (!ctx->check_flag) return FM_OK;
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  FM_HIP_TRY(ctx, hipStreamSynchronize((hipStream_t)stream));
  unsigned f = 0;
  FM_HIP_TRY(ctx, hipMemcpy(&f, ctx->check_flag, sizeof(unsigned), hipMemcpyDeviceToHost));
  if (!f) return FM_OK;
  FM_HIP_TRY(ctx, hipMemset(ctx->check_flag, 0, sizeof(unsigned)));
  FM_HIP_TRY(ctx, hipDeviceSynchronize());
  if (flags) *flags = f;
  return fm_fail(ctx, FM_EDEVICE_CHECK, "device check failed:%s%s%s%s",
                 (f & FM_CHECK_COORDS) ? " non-finite match coordinates;" : "",
                 (f & FM_CHECK_PARAMS) ? " non-finite pose parameters or essential matrices;" : "",
                 (f & FM_CHECK_DEGENERATE) ? " pairs with zero relative translation;" : "",
                 (f & FM_CHECK_LOSS) ? " non-finite loss or gradient;" : "");
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_check_finite(const T* __restrict__ p, int64_t n, unsigned bit,
                                                         unsigned* __restrict__ flag) {
  bool bad = false;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    bad = bad || !isfinite(p[k]);
  if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(flag, bit);
}

fm_status fm_check_finite(fm_ctx* ctx, hipStream_t st, const void* p, int64_t n, bool f64, unsigned bit) {
  if (!ctx->check || !p || n <= 0) return FM_OK;
  const int64_t want = grid_for(n, kBlock);
  const dim3 grid((unsigned)(want < 1024 ? want : 1024)), block(kBlock);
  if (f64)
    hipLaunchKernelGGL(k_check_finite<double>, grid, block, 0, st, (const double*)p, n, bit, ctx->check_flag);
  else
    hipLaunchKernelGGL(k_check_finite<float>, grid, block, 0, st, (const float*)p, n, bit, ctx->check_flag);
  FM_CHECK_LAUNCH(ctx);
  return FM_OK;
}

extern "C" const char* fm_last_error(const fm_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

// ------------------------------------------------------------------ kernels

// Bit 0: offsets not a valid CSR; bit 1: camera index out of range or i == j.
__global__ void k_validate(const int64_t* off, const int32_t* cams, int64_t P, int64_t M, int32_t N,
                           int* flag) {
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n > P) return;
  int bad = 0;
  int64_t a = off[n];
  if (n == 0 && a != 0) bad |= 1;
  if (n == P && a != M) bad |= 1;
  if (n < P) {
    int64_t b = off[n + 1];
    if (b < a || a < 0 || b > M) bad |= 1;
    int32_t i = cams[2 * n], j = cams[2 * n + 1];
    if (i < 0 || j < 0 || i >= N || j >= N || i == j) bad |= 2;
  }
  if (bad) atomicOr(flag, bad);
}

// Work items per pair (chunks of kChunk matches), written shifted by one so
// that an inclusive scan yields the exclusive offsets wi_off[0..P].
__global__ void k_wi_count(const int64_t* off, int64_t P, int64_t* wi_off) {
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n == 0) wi_off[0] = 0;
  if (n < P) {
    int64_t len = off[n + 1] - off[n];
    wi_off[n + 1] = (len + kChunk - 1) / kChunk;
  }
}

// In-place inclusive scan of x[0..n) by one block of 1024 threads: each
// thread scans a contiguous range serially, the range totals are scanned in
// LDS, and the ranges are offset.  Used only at scene set-up.
template <typename T>
__global__ __launch_bounds__(1024) void k_scan_inclusive(T* x, int64_t n) {
  __shared__ T tot[1024];
  const int tid = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t lo = tid * per;
  const int64_t hi = lo + per < n ? lo + per : n;
  T s = 0;
  for (int64_t k = lo; k < hi; ++k) {
    s += x[k];
    x[k] = s;
  }
  tot[tid] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    T v = tid >= d ? tot[tid - d] : 0;
    __syncthreads();
    tot[tid] += v;
    __syncthreads();
  }
  const T base = tid > 0 ? tot[tid - 1] : 0;
  for (int64_t k = lo; k < hi; ++k) x[k] += base;
}

__global__ void k_wi_fill(const int64_t* wi_off, int64_t P, int32_t* wi_pair) {
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < P)
    for (int64_t w = wi_off[n]; w < wi_off[n + 1]; ++w) wi_pair[w] = (int32_t)n;
}

__global__ void k_cam_degree(const int32_t* cams, int64_t P, int32_t* cam_ptr) {
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < P) {
    atomicAdd(&cam_ptr[cams[2 * n] + 1], 1);
    atomicAdd(&cam_ptr[cams[2 * n + 1] + 1], 1);
  }
}

__global__ void k_cam_scatter(const int32_t* cams, int64_t P, const int32_t* cam_ptr, int32_t* cursor,
                              int32_t* items) {
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < P) {
    for (int side = 0; side < 2; ++side) {
      int c = cams[2 * n + side];
      int pos = atomicAdd(&cursor[c], 1);
      items[cam_ptr[c] + pos] = (int32_t)(2 * n + side);
    }
  }
}

// Put every camera's incidence list in ascending item order (pair order), so
// that the per-camera gradient sums have a fixed order: each item's rank in
// its list is the number of smaller items in the list.
__global__ void k_cam_sort(const int32_t* cam_ptr, const int32_t* cam_of_slot, const int32_t* unsorted,
                           int64_t total, int32_t* sorted) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= total) return;
  int c = cam_of_slot[k];
  int lo = cam_ptr[c], hi = cam_ptr[c + 1];
  int v = unsorted[k];
  int rank = 0;
  for (int q = lo; q < hi; ++q) rank += unsorted[q] < v;
  sorted[lo + rank] = v;
}

// Inverse of the incidence lists: the position of every item in cam_items.
__global__ void k_pair_slots(const int32_t* cam_items, int64_t total, int32_t* pair_slot) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < total) pair_slot[cam_items[q]] = (int32_t)q;
}

__global__ void k_slot_camera(const int32_t* cam_ptr, int32_t N, int32_t* cam_of_slot) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < N)
    for (int q = cam_ptr[c]; q < cam_ptr[c + 1]; ++q) cam_of_slot[q] = c;
}

// ------------------------------------------------------------------ scene

static void scene_free(fm_scene* s) {
  if (!s) return;
  (void)hipFree(s->wi_off);
  (void)hipFree(s->wi_pair);
  (void)hipFree(s->multi);
  (void)hipFree(s->multi_first);
  (void)hipFree(s->big_pair);
  (void)hipFree(s->big_chunk);
  (void)hipFree(s->big_slot);
  (void)hipFree(s->groups);
  (void)hipFree(s->kept_slots);
  (void)hipFree(s->cam_ptr);
  (void)hipFree(s->cam_items);
  (void)hipFree(s->pair_slot);
  (void)hipFree(s->partials);
  (void)hipFree(s->ess);
  (void)hipFree(s->contrib);
  (void)hipFree(s->fo_rec);
  (void)hipFree(s->loss_part);
  (void)hipFree(s->rot);
  (void)hipFree(s->params_alt);
  (void)hipFree(s->bar);
  (void)hipFree(s->ta_rec);
  (void)hipFree(s->ta_part);
  (void)hipFree(s->ta_stats);
  (void)hipFree(s->ta_alt);
  (void)hipFree(s->lz);
  delete s;
}

extern "C" void fm_scene_destroy(fm_scene* s) { scene_free(s); }

extern "C" int64_t fm_scene_work_items(const fm_scene* s) { return s ? s->n_big + s->n_groups : -1; }

int fm_solve_coop_blocks(fm_ctx* ctx, bool cam);  // iterate.hip

template <typename T>
static hipError_t upload(T** dst, const std::vector<T>& v, hipStream_t st) {
  hipError_t e = hipMalloc(dst, sizeof(T) * (v.empty() ? 1 : v.size()));
  if (e == hipSuccess && !v.empty()) e = hipMemcpyAsync(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st);
  return e;
}

// Work decomposition of the Gram pass (make_gram_plan, host only): chunks of
// 64 big_rows(dtype) matches for pairs with more than small_max(dtype)
// matches, groups of four smaller pairs (pairs without matches included),
// both longest first; uploaded once per scene.
static fm_status build_gram_plan(fm_scene* s, hipStream_t st) {
  fm_ctx* ctx = s->ctx;
  const int64_t P = s->P;
  std::vector<int64_t> off(P + 1);
  hipError_t e = hipMemcpyAsync(off.data(), s->offsets, sizeof(int64_t) * (P + 1), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fm_fail(ctx, FM_EHIP, "gram plan: %s", hipGetErrorString(e));
  s->chunk = (int64_t)kLanes * big_rows(s->dtype);
  const GramPlan g = make_gram_plan(off.data(), P, kLanes, big_rows(s->dtype), small_max(s->dtype));
  s->n_big = (int64_t)g.big_pair.size();
  s->n_groups = (int64_t)g.groups.size() / 4;
  s->n_partials = g.n_partials;
  s->n_multi = g.n_multi;
  s->n_empty = g.n_empty;
  if ((e = upload(&s->big_pair, g.big_pair, st)) != hipSuccess ||
      (e = upload(&s->big_chunk, g.big_chunk, st)) != hipSuccess ||
      (e = upload(&s->big_slot, g.big_slot, st)) != hipSuccess ||
      (e = upload(&s->groups, g.groups, st)) != hipSuccess ||
      (e = upload(&s->multi, g.multi, st)) != hipSuccess || (e = upload(&s->multi_first, g.multi_first, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return fm_fail(ctx, e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EHIP, "gram plan: %s", hipGetErrorString(e));
  return FM_OK;
}

#define SCENE_TRY(expr)                                                                   \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess) {                                                               \
      (void)hipFree(tmp_i32);                                                             \
      (void)hipFree(flag);                                                                \
      scene_free(s);                                                                      \
      return fm_fail(ctx, _e == hipErrorOutOfMemory ? FM_ENOMEM : FM_EHIP, "%s: %s", #expr, \
                     hipGetErrorString(_e));                                              \
    }                                                                                     \
  } while (0)

extern "C" fm_status fm_scene_create(fm_ctx* ctx, int64_t P, int64_t M, int32_t N, const int64_t* off,
                                     const int32_t* cams, const void* uv, fm_dtype dtype,
                                     fm_stream stream_, fm_scene** out) {
  if (!ctx) return FM_EINVAL;
  if (!out) return fm_fail(ctx, FM_EINVAL, "fm_scene_create: out is NULL");
  *out = nullptr;
  if (P < 0 || M < 0 || N < 0) return fm_fail(ctx, FM_ESHAPE, "negative size (P=%lld M=%lld N=%d)", (long long)P, (long long)M, N);
  if (P > (int64_t)1 << 30 || N >= (1 << 30)) return fm_fail(ctx, FM_ESHAPE, "too many pairs or cameras");
  if (!off) return fm_fail(ctx, FM_EINVAL, "pair_offsets is NULL");
  if (P > 0 && !cams) return fm_fail(ctx, FM_EINVAL, "pair_cams is NULL");
  if (M > 0 && !uv) return fm_fail(ctx, FM_EINVAL, "uv is NULL");
  if (P > 0 && N < 2) return fm_fail(ctx, FM_ESHAPE, "pairs need at least two cameras");
  if (dtype != FM_F64 && dtype != FM_F32 && dtype != FM_BF16)
    return fm_fail(ctx, FM_EDTYPE, "unsupported coordinate dtype %d", (int)dtype);
  hipStream_t st = (hipStream_t)stream_;
  FM_HIP_TRY(ctx, hipSetDevice(ctx->device));
  fm_scene* s = new (std::nothrow) fm_scene();
  if (!s) return fm_fail(ctx, FM_ENOMEM, "host allocation failed");
  s->ctx = ctx;
  s->P = P; s->M = M; s->N = N;
  s->offsets = off; s->pair_cams = cams; s->uv = uv; s->dtype = dtype;
  int32_t* tmp_i32 = nullptr;
  int* flag = nullptr;
  SCENE_TRY(hipMalloc(&flag, sizeof(int)));
  SCENE_TRY(hipMemsetAsync(flag, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_validate, dim3(grid_for(P + 1, kBlock)), dim3(kBlock), 0, st, off, cams, P, M, N, flag);
  SCENE_TRY(hipGetLastError());
  int hflag = 0;
  SCENE_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  SCENE_TRY(hipStreamSynchronize(st));
  if (hflag) {
    (void)hipFree(flag);
    scene_free(s);
    return fm_fail(ctx, FM_ESHAPE, "%s%s", (hflag & 1) ? "pair_offsets is not a CSR over [0, M] " : "",
                   (hflag & 2) ? "pair_cams has an index out of [0, N) or i == j" : "");
  }
  // work items
  SCENE_TRY(hipMalloc(&s->wi_off, sizeof(int64_t) * (P + 1)));
  hipLaunchKernelGGL(k_wi_count, dim3(grid_for(P + 1, kBlock)), dim3(kBlock), 0, st, off, P, s->wi_off);
  SCENE_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_scan_inclusive<int64_t>, dim3(1), dim3(1024), 0, st, s->wi_off + 1, P);
  SCENE_TRY(hipGetLastError());
  SCENE_TRY(hipMemcpyAsync(&s->n_wi, s->wi_off + P, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  SCENE_TRY(hipStreamSynchronize(st));
  SCENE_TRY(hipMalloc(&s->wi_pair, sizeof(int32_t) * (s->n_wi > 0 ? s->n_wi : 1)));
  SCENE_TRY(hipMalloc(&s->kept_slots, sizeof(unsigned long long) * 16 * kKeptSlots));
  SCENE_TRY(hipMemsetAsync(s->kept_slots, 0, sizeof(unsigned long long) * 16 * kKeptSlots, st));
  if (P > 0) {
    hipLaunchKernelGGL(k_wi_fill, dim3(grid_for(P, kBlock)), dim3(kBlock), 0, st, s->wi_off, P, s->wi_pair);
    SCENE_TRY(hipGetLastError());
  }
  {
    fm_status prc = build_gram_plan(s, st);
    if (prc != FM_OK) {
      (void)hipFree(tmp_i32);
      (void)hipFree(flag);
      scene_free(s);
      return prc;
    }
  }
  // camera incidence lists
  SCENE_TRY(hipMalloc(&s->cam_ptr, sizeof(int32_t) * (N + 1)));
  SCENE_TRY(hipMalloc(&s->cam_items, sizeof(int32_t) * (2 * P + 1)));
  SCENE_TRY(hipMalloc(&s->pair_slot, sizeof(int32_t) * (2 * P + 1)));
  SCENE_TRY(hipMalloc(&tmp_i32, sizeof(int32_t) * (N + 1 + 4 * P + 2)));
  int32_t* cursor = tmp_i32;                 // [N+1]
  int32_t* unsorted = tmp_i32 + N + 1;       // [2P+1]
  int32_t* slot_cam = unsorted + 2 * P + 1;  // [2P+1]
  SCENE_TRY(hipMemsetAsync(s->cam_ptr, 0, sizeof(int32_t) * (N + 1), st));
  SCENE_TRY(hipMemsetAsync(cursor, 0, sizeof(int32_t) * (N + 1), st));
  if (P > 0) {
    hipLaunchKernelGGL(k_cam_degree, dim3(grid_for(P, kBlock)), dim3(kBlock), 0, st, cams, P, s->cam_ptr);
    SCENE_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_scan_inclusive<int32_t>, dim3(1), dim3(1024), 0, st, s->cam_ptr + 1, (int64_t)N);
    SCENE_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_cam_scatter, dim3(grid_for(P, kBlock)), dim3(kBlock), 0, st, cams, P, s->cam_ptr,
                       cursor, unsorted);
    SCENE_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_slot_camera, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, st, s->cam_ptr, N, slot_cam);
    SCENE_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_cam_sort, dim3(grid_for(2 * P, kBlock)), dim3(kBlock), 0, st, s->cam_ptr, slot_cam,
                       unsorted, 2 * P, s->cam_items);
    SCENE_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_pair_slots, dim3(grid_for(2 * P, kBlock)), dim3(kBlock), 0, st, s->cam_items, 2 * P,
                       s->pair_slot);
    SCENE_TRY(hipGetLastError());
  }
  SCENE_TRY(hipStreamSynchronize(st));
  (void)hipFree(tmp_i32);
  tmp_i32 = nullptr;
  (void)hipFree(flag);
  flag = nullptr;
  // workspace
  s->coop_blocks = fm_solve_coop_blocks(ctx, false);
  s->coop_blocks_cam = fm_solve_coop_blocks(ctx, true);
  if (s->coop_blocks <= 0 || s->coop_blocks_cam <= 0) {
    scene_free(s);
    return fm_fail(ctx, FM_ECOOP, "cannot size the cooperative solve kernel");
  }
  s->loss_part_cap = (int64_t)grid_for(P, kBlock);   // also covers k_pair_phase's blocks
  if (s->loss_part_cap < (int64_t)s->coop_blocks) s->loss_part_cap = s->coop_blocks;
  if (s->loss_part_cap < 2 * (int64_t)s->coop_blocks_cam) s->loss_part_cap = 2 * (int64_t)s->coop_blocks_cam;   // the camera loop double-buffers its partials
  SCENE_TRY(hipMalloc(&s->partials, sizeof(float) * 36 * (s->n_partials > 0 ? s->n_partials : 1)));
  SCENE_TRY(hipMalloc(&s->ess, sizeof(double) * 9 * (P > 0 ? P : 1)));
  SCENE_TRY(hipMalloc(&s->contrib, sizeof(float) * 24 * (P > 0 ? P : 1)));
  SCENE_TRY(hipMalloc(&s->fo_rec, sizeof(float) * 2 * (P > 0 ? P : 1)));
  SCENE_TRY(hipMalloc(&s->loss_part, sizeof(double) * s->loss_part_cap));
  SCENE_TRY(hipMalloc(&s->rot, sizeof(double) * 9 * 2 * (N > 0 ? N : 1)));
  SCENE_TRY(hipMalloc(&s->params_alt, sizeof(float) * 10 * (N > 0 ? N : 1)));
  SCENE_TRY(hipMalloc(&s->bar, sizeof(unsigned) * kBarWords));
  SCENE_TRY(hipMemsetAsync(s->bar, 0, sizeof(unsigned) * kBarWords, st));
  SCENE_TRY(hipStreamSynchronize(st));
  *out = s;
  return FM_OK;
}
