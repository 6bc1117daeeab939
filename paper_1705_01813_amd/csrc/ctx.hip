// Context, workspace, error handling and generic device primitives (fills,
// exclusive scan, deterministic float64 sum, the counter-based generator).
#include <cstdarg>
#include <cstring>

#include <vector>

#include "common.h"

knnkm_status knnkm_fail(knnkm_ctx* ctx, knnkm_status st, const char* fmt, ...) {
  if (!ctx) return st;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  ctx->err = buf;
  return st;
}

void* knnkm_ws(knnkm_ctx* ctx, const char* name, size_t bytes) {
  if (bytes == 0) bytes = 8;
  knnkm_buf& b = ctx->ws[name];
  if (b.bytes >= bytes) return b.ptr;
  if (ctx->capturing) {
    knnkm_fail(ctx, KNNKM_ENOMEM, "workspace '%s' would grow inside a graph capture", name);
    return nullptr;
  }
  // Stream-ordered: the old buffer is released after the work already queued
  // on the context stream, and growth never waits for other streams.
  if (b.ptr) {
    (void)hipFreeAsync(b.ptr, ctx->stream);
    b.ptr = nullptr;
    b.bytes = 0;
  }
  size_t want = bytes + bytes / 8;  // headroom against repeated growth
  void* p = nullptr;
  if (hipMallocAsync(&p, want, ctx->stream) != hipSuccess) {
    (void)hipGetLastError();
    knnkm_fail(ctx, KNNKM_ENOMEM, "workspace '%s': cannot allocate %zu bytes", name, want);
    return nullptr;
  }
  b.ptr = p;
  b.bytes = want;
  return p;
}

knnkm_status knnkm_ws_release(knnkm_ctx* ctx) {
  if (ctx->dry) return KNNKM_OK;
  for (auto& kv : ctx->ws)
    if (kv.second.ptr) (void)hipFreeAsync(kv.second.ptr, ctx->stream);
  ctx->ws.clear();
  ctx->fit_evals = nullptr;
  ctx->fit_actives = nullptr;
  ctx->fit_moved = nullptr;
  for (auto& pl : ctx->tm_plan) {  // their device tables were workspace
    tm_plan_free(pl);
    pl = nullptr;
  }
  KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return KNNKM_OK;
}

knnkm_status knnkm_check(knnkm_ctx* ctx, const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    ctx->sticky = true;
    return knnkm_fail(ctx, KNNKM_EDEVICE, "%s: %s", where, hipGetErrorString(e));
  }
  return KNNKM_OK;
}

// Message of the last failed call that had no context (knnkm_create).
static thread_local std::string g_create_err;

extern "C" knnkm_status knnkm_create(int device, void* hip_stream, knnkm_ctx** out) {
  if (!out) {
    g_create_err = "knnkm_create: out is null";
    return KNNKM_EINVAL;
  }
  *out = nullptr;
  knnkm_ctx* ctx = new (std::nothrow) knnkm_ctx();
  if (!ctx) return KNNKM_ENOMEM;
  ctx->device = device;
  ctx->dry = device < 0;
  ctx->stream = (hipStream_t)hip_stream;
  if (!ctx->dry) {
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || device >= ndev) {
      char buf[256];
      snprintf(buf, sizeof(buf), "knnkm_create: device %d unavailable (%d devices, %s)", device, ndev,
               hipGetErrorString(e));
      g_create_err = buf;
      (void)hipGetLastError();
      delete ctx;
      return KNNKM_EDEVICE;
    }
    e = hipSetDevice(device);
    if (e != hipSuccess) {
      g_create_err = std::string("knnkm_create: hipSetDevice: ") + hipGetErrorString(e);
      delete ctx;
      return KNNKM_EDEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cus = prop.multiProcessorCount;
    // device address of the fixed scratch used by the allocation-free calls
    if (ks_noalloc_setup(ctx) != KNNKM_OK) {
      g_create_err = ctx->err;
      delete ctx;
      return KNNKM_EDEVICE;
    }
  }
  *out = ctx;
  return KNNKM_OK;
}

extern "C" knnkm_status knnkm_destroy(knnkm_ctx* ctx) {
  if (!ctx) return KNNKM_EINVAL;
  if (!ctx->dry) {
    (void)hipSetDevice(ctx->device);
    for (auto& kv : ctx->ws)
      if (kv.second.ptr) (void)hipFreeAsync(kv.second.ptr, ctx->stream);
    (void)hipStreamSynchronize(ctx->stream);
  }
  for (auto* pl : ctx->tm_plan) tm_plan_free(pl);
  for (hipEvent_t e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  for (hipEvent_t e : ctx->tune_ev)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
  return KNNKM_OK;
}

extern "C" knnkm_status knnkm_set_stream(knnkm_ctx* ctx, void* hip_stream) {
  if (!ctx) return KNNKM_EINVAL;
  // workspace buffers are stream-ordered allocations of the old stream
  if (!ctx->dry && ctx->stream != (hipStream_t)hip_stream) {
    (void)hipSetDevice(ctx->device);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
      ctx->sticky = true;
      return knnkm_fail(ctx, KNNKM_EDEVICE, "knnkm_set_stream: synchronising the old stream failed");
    }
  }
  ctx->stream = (hipStream_t)hip_stream;
  return KNNKM_OK;
}

extern "C" const char* knnkm_last_error(const knnkm_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

extern "C" knnkm_status knnkm_default_params(knnkm_params* p) {
  if (!p) return KNNKM_EINVAL;
  memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(knnkm_params);
  p->kappa = 50;
  p->xi = 50;
  p->tau = 10;
  p->bisect_iters = 2;
  p->precision = KNNKM_FP32;
  p->init = KNNKM_INIT_TWOMEANS;
  p->max_iters = 30;
  p->early_stop = 0;
  p->seed = 0;
  return KNNKM_OK;
}

extern "C" knnkm_status knnkm_workspace_bytes(const knnkm_ctx* ctx, int64_t* out) {
  if (!ctx || !out) return KNNKM_EINVAL;
  int64_t s = 0;
  for (auto& kv : ctx->ws) s += (int64_t)kv.second.bytes;
  *out = s;
  return KNNKM_OK;
}

hipEvent_t knnkm_event(knnkm_ctx* ctx, int i) {
  if ((int)ctx->ev.size() <= i) ctx->ev.resize(i + 1, nullptr);
  if (!ctx->ev[i] && hipEventCreate(&ctx->ev[i]) != hipSuccess) {
    (void)hipGetLastError();
    ctx->ev[i] = nullptr;
  }
  return ctx->ev[i];
}

extern "C" knnkm_status knnkm_enable_graphs(knnkm_ctx* ctx, int32_t on) {
  if (!ctx) return KNNKM_EINVAL;
  ctx->graphs = on != 0;
  return KNNKM_OK;
}

extern "C" knnkm_status knnkm_enable_timing(knnkm_ctx* ctx, int32_t on) {
  if (!ctx) return KNNKM_EINVAL;
  ctx->timing = on < 0 ? 0 : (on > 2 ? 2 : on);
  ctx->build_ev = ctx->fit_ev = ctx->assign_ev0 = -1;
  ctx->assign_n = 0;
  ctx->fit_iters = 0;
  return KNNKM_OK;
}

static double ev_ms(knnkm_ctx* ctx, int a) {
  float ms = 0.f;
  if (a < 0 || a + 1 >= (int)ctx->ev.size() || !ctx->ev[a] || !ctx->ev[a + 1]) return -1.0;
  if (hipEventSynchronize(ctx->ev[a + 1]) != hipSuccess) return -1.0;
  if (hipEventElapsedTime(&ms, ctx->ev[a], ctx->ev[a + 1]) != hipSuccess) return -1.0;
  return (double)ms;
}

extern "C" knnkm_status knnkm_phase_times(knnkm_ctx* ctx, double* out, int32_t count) {
  if (!ctx || !out || count < 1) return KNNKM_EINVAL;
  double v[8] = {-1.0, -1.0, -1.0, -1.0, 0.0, 0.0, -1.0, -1.0};
  if (!ctx->dry) {
    (void)hipSetDevice(ctx->device);
    v[0] = ev_ms(ctx, ctx->build_ev);
    v[1] = ev_ms(ctx, ctx->fit_ev);
    v[2] = ev_ms(ctx, ctx->fit_ev + 1);
    if (ctx->assign_ev0 >= 0) {
      double s = 0.0;
      for (int j = 0; j < ctx->assign_n; ++j) s += ev_ms(ctx, ctx->assign_ev0 + 2 * j);
      v[3] = s;
    }
    v[4] = ctx->fit_ev >= 0 ? (double)ctx->fit_iters : 0.0;
    v[5] = (double)ctx->assign_n;
    const int64_t* per_sweep[2] = {ctx->fit_evals, ctx->fit_actives};
    for (int c = 0; c < 2; ++c) {
      if (!per_sweep[c] || ctx->assign_n <= 0 || count <= 6 + c) continue;
      std::vector<int64_t> ev((size_t)ctx->assign_n);
      if (hipMemcpyAsync(ev.data(), per_sweep[c] + 1, sizeof(int64_t) * ev.size(), hipMemcpyDeviceToHost,
                         ctx->stream) == hipSuccess &&
          hipStreamSynchronize(ctx->stream) == hipSuccess) {
        double s = 0.0;
        for (int64_t e : ev) s += (double)e;
        v[6 + c] = s;
      } else {
        (void)hipGetLastError();
      }
    }
  }
  for (int i = 0; i < count && i < 8; ++i) out[i] = v[i];
  for (int i = 8; i < count; ++i) out[i] = 0.0;
  return KNNKM_OK;
}

extern "C" knnkm_status knnkm_sweep_stats(knnkm_ctx* ctx, double* assign_ms, int64_t* listed, int64_t* evaluated,
                                         int64_t* moved, int32_t count, int32_t* n_out) {
  if (!ctx || count < 0 || !n_out) return KNNKM_EINVAL;
  *n_out = 0;
  if (ctx->dry) return KNNKM_OK;
  (void)hipSetDevice(ctx->device);
  const int ns = std::min(count, ctx->fit_iters);
  if (ns <= 0) return KNNKM_OK;
  for (int j = 0; j < ns; ++j) {
    if (assign_ms) assign_ms[j] = (ctx->assign_ev0 >= 0 && j < ctx->assign_n) ? ev_ms(ctx, ctx->assign_ev0 + 2 * j) : -1.0;
  }
  const int64_t* src[3] = {ctx->fit_actives, ctx->fit_evals, ctx->fit_moved};
  int64_t* dst[3] = {listed, evaluated, moved};
  for (int c = 0; c < 3; ++c) {
    if (!dst[c]) continue;
    for (int j = 0; j < ns; ++j) dst[c][j] = -1;
    if (!src[c]) continue;
    if (hipMemcpyAsync(dst[c], src[c] + 1, sizeof(int64_t) * (size_t)ns, hipMemcpyDeviceToHost, ctx->stream) !=
            hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
      (void)hipGetLastError();
      return knnkm_fail(ctx, KNNKM_EDEVICE, "sweep_stats: copy failed");
    }
  }
  *n_out = ns;
  return KNNKM_OK;
}

// ------------------------------------------------------------------ fills --
__global__ void k_fill_i64(int64_t* p, int64_t count, int64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
knnkm_status ks_fill_i64(knnkm_ctx* ctx, int64_t* p, int64_t count, int64_t v) {
  if (count <= 0) return KNNKM_OK;
  k_fill_i64<<<grid_for(count, 256, 4096), 256, 0, ctx->stream>>>(p, count, v);
  return knnkm_check(ctx, "fill_i64");
}
knnkm_status ks_fill_i32(knnkm_ctx* ctx, int32_t* p, int64_t count, int32_t v) {
  if (count <= 0) return KNNKM_OK;
  k_fill_i32<<<grid_for(count, 256, 4096), 256, 0, ctx->stream>>>(p, count, v);
  return knnkm_check(ctx, "fill_i32");
}

// ------------------------------------------------------- exclusive scan --
// Tiles of SCAN_TILE values per 256-thread block; tile totals are scanned
// recursively, then added back.
#define SCAN_TILE 1024

__global__ __launch_bounds__(256) void k_scan_tiles(const int32_t* in, int32_t* out, int64_t count,
                                                    int32_t* tile_sums) {
  __shared__ int32_t sh[8];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * 4;
  int32_t v[4];
  int32_t s = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    v[j] = (base + j < count) ? in[base + j] : 0;
    s += v[j];
  }
  int32_t tot;
  int32_t ex = block_scan_excl_256(s, sh, &tot);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (base + j < count) out[base + j] = ex;
    ex += v[j];
  }
  if (threadIdx.x == 0 && tile_sums) tile_sums[blockIdx.x] = tot;
}

__global__ void k_scan_add(int32_t* out, int64_t count, const int32_t* tile_offsets) {
  int64_t i = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * 4;
  int32_t add = tile_offsets[blockIdx.x];
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (i + j < count) out[i + j] += add;
}

__global__ void k_write_total(const int32_t* in, const int32_t* out, int64_t count, int32_t* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = (count ? out[count - 1] + in[count - 1] : 0);
}

static knnkm_status scan_rec(knnkm_ctx* ctx, const int32_t* in, int32_t* out, int64_t count,
                             int depth) {
  int64_t tiles = (count + SCAN_TILE - 1) / SCAN_TILE;
  if (tiles <= 1) {
    k_scan_tiles<<<1, 256, 0, ctx->stream>>>(in, out, count, nullptr);
    return knnkm_check(ctx, "scan");
  }
  char name[32];
  snprintf(name, sizeof(name), "scan_sums%d", depth);
  KNNKM_WS(ctx, sums, int32_t, name, tiles + 1);
  k_scan_tiles<<<(unsigned)tiles, 256, 0, ctx->stream>>>(in, out, count, sums);
  KNNKM_TRY(knnkm_check(ctx, "scan tiles"));
  KNNKM_TRY(scan_rec(ctx, sums, sums, tiles, depth + 1));
  k_scan_add<<<(unsigned)tiles, 256, 0, ctx->stream>>>(out, count, sums);
  return knnkm_check(ctx, "scan add");
}

knnkm_status ks_scan_exclusive(knnkm_ctx* ctx, const int32_t* in, int32_t* out, int64_t count,
                               bool with_total) {
  if (count <= 0) {
    if (with_total) return ks_fill_i32(ctx, out, 1, 0);
    return KNNKM_OK;
  }
  // The total needs the last input value, which an in-place scan overwrites.
  if (with_total) {
    KNNKM_WS(ctx, last, int32_t, "scan_last", 1);
    hipMemcpyAsync(last, in + count - 1, sizeof(int32_t), hipMemcpyDeviceToDevice, ctx->stream);
    KNNKM_TRY(scan_rec(ctx, in, out, count, 0));
    k_write_total<<<1, 64, 0, ctx->stream>>>(last, out + count - 1, 1, out + count);
    return knnkm_check(ctx, "scan total");
  }
  return scan_rec(ctx, in, out, count, 0);
}

// ------------------------------------------------ deterministic f64 sum --
// Each of 256 threads sums a fixed strided subset in order; the block then
// combines the 256 partials in a fixed tree.  Same order on every run.
__global__ __launch_bounds__(256) void k_sum_f64(const double* in, int64_t count, double* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) s += in[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

__global__ __launch_bounds__(256) void k_sum_f64_tiles(const double* in, int64_t count,
                                                       double* partial) {
  __shared__ double sh[256];
  int64_t base = (int64_t)blockIdx.x * 8192;
  double s = 0.0;
  for (int j = threadIdx.x; j < 8192; j += 256)
    if (base + j < count) s += in[base + j];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

knnkm_status ks_sum_f64_with(knnkm_ctx* ctx, const double* in, int64_t count, double* part, double* out) {
  if (count > 65536) {
    const int64_t tiles = (count + 8191) / 8192;
    k_sum_f64_tiles<<<(unsigned)tiles, 256, 0, ctx->stream>>>(in, count, part);
    KNNKM_TRY(knnkm_check(ctx, "sum_f64 tiles"));
    k_sum_f64<<<1, 256, 0, ctx->stream>>>(part, tiles, out);
    return knnkm_check(ctx, "sum_f64");
  }
  k_sum_f64<<<1, 256, 0, ctx->stream>>>(in, count, out);
  return knnkm_check(ctx, "sum_f64");
}

knnkm_status ks_sum_f64(knnkm_ctx* ctx, const double* in, int64_t count, double* out) {
  double* part = nullptr;
  if (count > 65536) {
    KNNKM_WS(ctx, p, double, "sum_f64_part", (count + 8191) / 8192);
    part = p;
  }
  return ks_sum_f64_with(ctx, in, count, part, out);
}

// --------------------------------------------------- generator exposure --
__global__ void k_rng_draw(uint64_t key, uint64_t ctr0, int64_t count, uint64_t* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = sm_draw(key, ctr0 + (uint64_t)i);
}

extern "C" knnkm_status knnkm_rng_draw(knnkm_ctx* ctx, uint64_t seed, uint64_t stream,
                                       uint64_t ctr0, int64_t count, uint64_t* out) {
  if (!ctx) return KNNKM_EINVAL;
  if (count < 0 || (count > 0 && !out)) return knnkm_fail(ctx, KNNKM_EINVAL, "rng_draw: bad args");
  if (ctx->sticky) return KNNKM_EDEVICE;
  if (ctx->dry || count == 0) return KNNKM_OK;
  k_rng_draw<<<grid_for(count, 256, 4096), 256, 0, ctx->stream>>>(sm_key(seed, stream), ctr0, count,
                                                                   out);
  return knnkm_check(ctx, "rng_draw");
}
