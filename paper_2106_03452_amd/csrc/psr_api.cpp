// C ABI of the solver library: argument checking, context (twiddle tables,
// options, stage timers), workspace and saved-state layout, dispatch to the
// per-resolution launch sequences.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "psr.h"
#include "psr_internal.h"
#include "psr_mc.h"
#include "psr_opt.h"
#include "psr_slab.h"

namespace psr {

struct cf {
  float x, y;
};

struct Timers {
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t open[NUM_STAGES] = {};
  double ms[NUM_STAGES] = {};
  int64_t cnt[NUM_STAGES] = {};
  uint32_t mask = 0xffffffffu;  // stages to time

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void flush() {
    for (auto& r : pending) {
      float t = 0.0f;
      if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        ms[r.stage] += t;
        cnt[r.stage] += 1;
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  ~Timers() {
    flush();
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

void timer_begin(Timers* t, int stage, hipStream_t s) {
  if (!((t->mask >> stage) & 1u)) return;
  hipEvent_t e = t->get();
  if (!e) return;
  (void)hipEventRecord(e, s);
  t->open[stage] = e;
}

void timer_end(Timers* t, int stage, hipStream_t s) {
  hipEvent_t a = t->open[stage];
  if (!a) return;
  hipEvent_t b = t->get();
  if (!b) return;
  (void)hipEventRecord(b, s);
  t->open[stage] = nullptr;
  t->pending.push_back({stage, a, b});
  if (t->pending.size() > 8192) t->flush();
}

}  // namespace psr

struct psr_ctx {
  int device = 0;
  psr::cf* tw = nullptr;
  double m = 0.5;
  int reading = 0;
  psr::Timers* timers = nullptr;
  // device address of this device's static scratch array (psr_forward_static)
  void* scratch = nullptr;
  // point-source tables of the backward, one per (res, sigma), kept until
  // the context is destroyed
  struct KTab {
    int res;
    float sigma;
    float* table;
  };
  std::mutex kmu;
  std::vector<KTab> ktabs;
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

bool valid_res(int res) {
  return res >= PSR_MIN_RES && res <= PSR_MAX_RES && (res & (res - 1)) == 0;
}

bool valid_P(int64_t P) { return P >= 1 && P <= ((int64_t)1 << 30); }

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

psr::JobArg make_job(const float* pts, const float* nrm, int64_t P, float sigma, float* chi, void* saved, void* ws) {
  psr::JobArg j;
  j.pts = pts;
  j.nrm = nrm;
  j.chi = chi;
  j.dchi = nullptr;
  j.dpts = nullptr;
  j.dnrm = nullptr;
  j.ws = ws;
  j.sv = saved;
  j.aux_in = nullptr;
  j.aux_out = nullptr;
  j.ktab = nullptr;
  j.P = P;
  j.sigma = sigma;
  j.pad = 0;
  return j;
}

bool valid_slab(int res, int slabs) {
  return res >= psr::kSlabMinRes && res <= psr::kSlabMaxRes && (res & (res - 1)) == 0 && slabs >= 1 &&
         slabs <= psr::kMaxSlabs && slabs <= res && (slabs & (slabs - 1)) == 0;
}

static_assert(sizeof(psr_slab_result) == sizeof(psr::SlabResult) &&
                  offsetof(psr_slab_result, chi0) == offsetof(psr::SlabResult, chi0) &&
                  offsetof(psr_slab_result, status) == offsetof(psr::SlabResult, status),
              "psr_slab_result and the kernels' SlabResult share one layout");

psr::SlabArgs slab_args(psr_ctx* ctx, const psr::SlabLayout& L, void* ws, int64_t P, float sigma, int slabs,
                        float* chi) {
  char* b = static_cast<char*>(ws);
  psr::SlabArgs a{};
  a.tw = ctx->tw;
  a.chi = chi;
  a.hdr = reinterpret_cast<psr::SlabHeader*>(b + L.hdr);
  a.counts = reinterpret_cast<int*>(b + L.counts);
  a.off = reinterpret_cast<int*>(b + L.off);
  a.bsum = reinterpret_cast<int*>(b + L.bsum);
  a.tmp = reinterpret_cast<psr::PointRec*>(b + L.tmp);
  a.colrank = reinterpret_cast<int2*>(b + L.colrank);
  a.sorted = reinterpret_cast<psr::PointRec*>(b + L.sorted);
  a.val = reinterpret_cast<double*>(b + L.val);
  a.red = reinterpret_cast<double*>(b + L.red);
  a.A = reinterpret_cast<psr::cf*>(b + L.A);
  a.X = reinterpret_cast<psr::cf*>(b + L.X);
  a.Z = reinterpret_cast<psr::cf*>(b + L.Z);
  a.halo = reinterpret_cast<float*>(b + L.halo);
  a.P = P;
  a.sigma = sigma;
  a.m = (float)ctx->m;
  a.reading = ctx->reading;
  a.G = slabs;
  return a;
}

psr::Exec make_exec(psr_ctx* ctx, hipStream_t stream) {
  psr::Exec x;
  x.stream = stream;
  x.tw = ctx->tw;
  x.m = ctx->m;
  x.reading = ctx->reading;
  x.timers = ctx->timers;
  return x;
}

// The backward's point-source table of (res, sigma): built on first use,
// in FP64 on `stream` (a one-time allocation of the table and of its build
// scratch, then a synchronisation of `stream` so that every stream may read
// it), then reused.
int point_source_table(psr_ctx* ctx, int res, float sigma, hipStream_t stream, const float** out) {
  std::lock_guard<std::mutex> lk(ctx->kmu);
  for (const auto& k : ctx->ktabs) {
    if (k.res == res && k.sigma == sigma) {
      *out = k.table;
      return PSR_OK;
    }
  }
  float* table = nullptr;
  void* scratch = nullptr;
  if (hipMalloc(&table, psr::ktab_floats(res) * sizeof(float)) != hipSuccess) return PSR_ENOMEM;
  if (hipMalloc(&scratch, psr::ktab_scratch_bytes(res)) != hipSuccess) {
    (void)hipFree(table);
    return PSR_ENOMEM;
  }
  int rc = psr::build_point_source_table(res, sigma, table, scratch, stream) ? PSR_EDEVICE : PSR_OK;
  if (hipStreamSynchronize(stream) != hipSuccess) rc = PSR_EDEVICE;
  (void)hipFree(scratch);
  if (rc) {
    (void)hipFree(table);
    return rc;
  }
  ctx->ktabs.push_back({res, sigma, table});
  *out = table;
  return PSR_OK;
}

const char* const kStageNames[psr::NUM_STAGES] = {
    "bin", "P1_splat_r2c", "P2_fft_j1", "P3_fft_j0_spectral_ifft_j0", "P4_ifft_j1", "P5_c2r_gather",
    "fwd_reduce", "normalize", "bwd_reduce", "B1_cotangent_r2c", "B2_fft_j1", "B3_fft_j0_conjop_ifft_j0",
    "B4_ifft_j1", "B5_c2r_gather", "bwd_finalize", "P12_splat_r2c_fft_j1", "P45_ifft_j1_c2r_gather",
    "B12_cotangent_r2c_fft_j1", "B45_ifft_j1_c2r_gather", "B1a_reduce_r2c", "slab_bin", "S1_splat_r2c",
    "S2_fft_j1_exchange", "S3_pencil_fft_j0_spectral", "S4_ifft_k1", "S5_c2r_halo", "slab_gather_mean",
    "slab_normalize"};

}  // namespace

extern "C" {

int psr_version(void) { return 10000; }

const char* psr_strerror(int code) {
  switch (code) {
    case PSR_OK: return "ok";
    case PSR_EINVAL: return "invalid argument";
    case PSR_ENOMEM: return "out of device memory";
    case PSR_EDEGENERATE: return "degenerate scale: chi'(0) - mean is zero or non-finite";
    case PSR_EDEVICE: return "HIP runtime error";
    case PSR_ENOTREADY: return "not ready";
    case PSR_ENONFINITE: return "non-finite point coordinate";
    case PSR_ETOOBIG: return "problem too large for this entry point";
    default: return "unknown status code";
  }
}

int psr_ctx_create(psr_ctx** out, int device) {
  if (!out) return PSR_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) return PSR_EDEVICE;
  if (device < 0 || device >= ndev) return PSR_EINVAL;
  DeviceGuard g(device);
  psr_ctx* c = new (std::nothrow) psr_ctx();
  if (!c) return PSR_ENOMEM;
  c->device = device;
  // twiddle tables exp(-2 pi i e / L), e in [0, L), built in FP64, for L = 2..1024
  const int total = 2048;
  std::vector<psr::cf> host(total, psr::cf{0.0f, 0.0f});
  for (int L = 2; L <= 1024; L *= 2) {
    for (int e = 0; e < L; ++e) {
      const double a = -2.0 * M_PI * (double)e / (double)L;
      host[L + e] = psr::cf{(float)std::cos(a), (float)std::sin(a)};
    }
  }
  if (hipMalloc(&c->tw, total * sizeof(psr::cf)) != hipSuccess) {
    delete c;
    return PSR_ENOMEM;
  }
  if (hipMemcpy(c->tw, host.data(), total * sizeof(psr::cf), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(c->tw);
    delete c;
    return PSR_EDEVICE;
  }
  // this device's copy of the static scratch array (device current here);
  // without it only psr_forward_static is unavailable
  if (psr::static_scratch_address(&c->scratch) != 0) c->scratch = nullptr;
  *out = c;
  return PSR_OK;
}

int psr_ctx_destroy(psr_ctx* ctx) {
  if (!ctx) return PSR_EINVAL;
  DeviceGuard g(ctx->device);
  delete ctx->timers;
  if (ctx->tw) (void)hipFree(ctx->tw);
  for (auto& k : ctx->ktabs) (void)hipFree(k.table);
  delete ctx;
  return PSR_OK;
}

int psr_ctx_set(psr_ctx* ctx, const char* key, double value) {
  if (!ctx || !key) return PSR_EINVAL;
  if (!std::strcmp(key, "m")) {
    if (!(value > 0.0) || !std::isfinite(value)) return PSR_EINVAL;
    ctx->m = value;
    return PSR_OK;
  }
  if (!std::strcmp(key, "reading")) {
    if (value != 0.0 && value != 1.0) return PSR_EINVAL;
    ctx->reading = (int)value;
    return PSR_OK;
  }
  if (!std::strcmp(key, "timers")) {
    if (value != 0.0 && value != 1.0) return PSR_EINVAL;
    DeviceGuard g(ctx->device);
    if (value == 1.0 && !ctx->timers) {
      ctx->timers = new (std::nothrow) psr::Timers();
      if (!ctx->timers) return PSR_ENOMEM;
    }
    if (value == 0.0 && ctx->timers) {
      delete ctx->timers;
      ctx->timers = nullptr;
    }
    return PSR_OK;
  }
  if (!std::strcmp(key, "timer_mask")) {
    if (!ctx->timers || !(value >= 0.0) || value > 4294967295.0 || value != std::floor(value)) return PSR_EINVAL;
    ctx->timers->mask = (uint32_t)value;
    return PSR_OK;
  }
  return PSR_EINVAL;
}

int psr_ctx_get(const psr_ctx* ctx, const char* key, double* value) {
  if (!ctx || !key || !value) return PSR_EINVAL;
  if (!std::strcmp(key, "m")) *value = ctx->m;
  else if (!std::strcmp(key, "reading")) *value = ctx->reading;
  else if (!std::strcmp(key, "timers")) *value = ctx->timers ? 1.0 : 0.0;
  else if (!std::strcmp(key, "device")) *value = ctx->device;
  else if (!std::strcmp(key, "timer_mask")) *value = ctx->timers ? (double)ctx->timers->mask : 0.0;
  else return PSR_EINVAL;
  return PSR_OK;
}

int psr_workspace_bytes(int res, int64_t npoints, int with_backward, size_t* bytes) {
  (void)with_backward;
  if (!bytes || !valid_res(res) || !valid_P(npoints)) return PSR_EINVAL;
  *bytes = psr::ws_layout(res, npoints).total;
  return PSR_OK;
}

int psr_saved_bytes(int res, int64_t npoints, size_t* bytes) {
  if (!bytes || !valid_res(res) || !valid_P(npoints)) return PSR_EINVAL;
  *bytes = psr::saved_layout(res, npoints).total;
  return PSR_OK;
}

int psr_forward(psr_ctx* ctx, const float* points, const float* normals, int64_t npoints, int res, float sigma,
                float* chi, void* saved, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!ctx || !points || !normals || !chi || !saved || !workspace) return PSR_EINVAL;
  if (!valid_res(res) || !valid_P(npoints) || !(sigma >= 0.0f) || !std::isfinite(sigma)) return PSR_EINVAL;
  if (!aligned(saved, 256) || !aligned(workspace, 256) || !aligned(chi, 16)) return PSR_EINVAL;
  if (workspace_bytes < psr::ws_layout(res, npoints).total) return PSR_EINVAL;
  DeviceGuard g(ctx->device);
  psr::Exec x = make_exec(ctx, stream);
  psr::JobArg j = make_job(points, normals, npoints, sigma, chi, saved, workspace);
  return psr::run_jobs(x, res, &j, 1, psr::RUN_FORWARD);
}

int psr_forward_static(psr_ctx* ctx, const float* points, const float* normals, int64_t npoints, int res,
                       float sigma, float* chi, hipStream_t stream) {
  if (!ctx || !points || !normals || !chi) return PSR_EINVAL;
  if (!valid_res(res) || !valid_P(npoints) || !(sigma >= 0.0f) || !std::isfinite(sigma)) return PSR_EINVAL;
  if (!aligned(chi, 16)) return PSR_EINVAL;
  const size_t sv_bytes = psr::saved_layout(res, npoints).total;  // a multiple of 256
  if (sv_bytes + psr::ws_layout(res, npoints).total > psr::kStaticScratchBytes) return PSR_ETOOBIG;
  if (!ctx->scratch) return PSR_EDEVICE;
  DeviceGuard g(ctx->device);
  psr::Exec x = make_exec(ctx, stream);
  x.timers = nullptr;  // no event creation on this path
  char* base = static_cast<char*>(ctx->scratch);
  psr::JobArg j = make_job(points, normals, npoints, sigma, chi, base, base + sv_bytes);
  return psr::run_jobs(x, res, &j, 1, psr::RUN_FORWARD);
}

int psr_backward(psr_ctx* ctx, int64_t npoints, int res, float sigma, const float* chi, const void* saved,
                 const float* dchi, float* dpoints, float* dnormals, void* workspace, size_t workspace_bytes,
                 hipStream_t stream) {
  if (!ctx || !chi || !saved || !dchi || !workspace) return PSR_EINVAL;
  if (!valid_res(res) || !valid_P(npoints) || !(sigma >= 0.0f) || !std::isfinite(sigma)) return PSR_EINVAL;
  if (!aligned(saved, 256) || !aligned(workspace, 256) || !aligned(chi, 16) || !aligned(dchi, 16))
    return PSR_EINVAL;
  if (workspace_bytes < psr::ws_layout(res, npoints).total) return PSR_EINVAL;
  DeviceGuard g(ctx->device);
  const float* kt = nullptr;
  if (int rc = point_source_table(ctx, res, sigma, stream, &kt)) return rc;
  psr::Exec x = make_exec(ctx, stream);
  psr::JobArg j = make_job(nullptr, nullptr, npoints, sigma, const_cast<float*>(chi), const_cast<void*>(saved),
                           workspace);
  j.ktab = kt;
  j.dchi = dchi;
  j.dpts = dpoints;
  j.dnrm = dnormals;
  return psr::run_jobs(x, res, &j, 1, psr::RUN_BACKWARD);
}

int psr_slab_workspace_bytes(int res, int64_t npoints, int slabs, size_t* bytes) {
  if (!bytes || !valid_slab(res, slabs) || npoints < 0 || npoints > ((int64_t)1 << 30)) return PSR_EINVAL;
  *bytes = psr::slab_layout(res, npoints, slabs).total;
  return PSR_OK;
}

int psr_slab_forward(psr_ctx* ctx, const float* points, const float* normals, int64_t npoints, int res, float sigma,
                     int slabs, float* chi, psr_slab_result* result, void* workspace, size_t workspace_bytes,
                     hipStream_t stream) {
  if (!ctx || !points || !normals || !chi || !result || !workspace) return PSR_EINVAL;
  if (!valid_slab(res, slabs) || !valid_P(npoints) || !(sigma >= 0.0f) || !std::isfinite(sigma)) return PSR_EINVAL;
  if (!aligned(workspace, 256) || !aligned(chi, 16) || !aligned(result, 8)) return PSR_EINVAL;
  const psr::SlabLayout L = psr::slab_layout(res, npoints, slabs);
  if (workspace_bytes < L.total) return PSR_EINVAL;
  DeviceGuard g(ctx->device);
  psr::Exec x = make_exec(ctx, stream);
  psr::SlabArgs a = slab_args(ctx, L, workspace, npoints, sigma, slabs, chi);
  a.pts = points;
  a.nrm = normals;
  a.result = reinterpret_cast<psr::SlabResult*>(result);
  return psr::run_slab(x, res, a) ? PSR_EDEVICE : PSR_OK;
}

int psr_slab_debug_spectral(psr_ctx* ctx, const float* field, int res, float sigma, int slabs, float* chi_prime,
                            void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!ctx || !field || !chi_prime || !workspace) return PSR_EINVAL;
  if (!valid_slab(res, slabs) || !(sigma >= 0.0f) || !std::isfinite(sigma)) return PSR_EINVAL;
  if (!aligned(workspace, 256) || !aligned(chi_prime, 16) || !aligned(field, 16)) return PSR_EINVAL;
  const psr::SlabLayout L = psr::slab_layout(res, 0, slabs);
  if (workspace_bytes < L.total) return PSR_EINVAL;
  DeviceGuard g(ctx->device);
  psr::Exec x = make_exec(ctx, stream);
  psr::SlabArgs a = slab_args(ctx, L, workspace, 0, sigma, slabs, chi_prime);
  a.field = field;
  return psr::run_slab(x, res, a) ? PSR_EDEVICE : PSR_OK;
}

int psr_ctx_prepare(psr_ctx* ctx, int res, float sigma, hipStream_t stream) {
  if (!ctx || !valid_res(res) || !(sigma >= 0.0f) || !std::isfinite(sigma)) return PSR_EINVAL;
  DeviceGuard g(ctx->device);
  const float* kt = nullptr;
  return point_source_table(ctx, res, sigma, stream, &kt);
}

int psr_saved_status(const void* saved, hipStream_t stream, int* status) {
  if (!saved || !status) return PSR_EINVAL;
  if (hipStreamSynchronize(stream) != hipSuccess) return PSR_EDEVICE;
  psr::SavedHeader h;
  if (hipMemcpy(&h, saved, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return PSR_EDEVICE;
  *status = h.status;
  return PSR_OK;
}

int psr_saved_scalars(const void* saved, hipStream_t stream, double* mean, double* cscale, double* scale,
                      double* chi0) {
  if (!saved) return PSR_EINVAL;
  if (hipStreamSynchronize(stream) != hipSuccess) return PSR_EDEVICE;
  psr::SavedHeader h;
  if (hipMemcpy(&h, saved, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return PSR_EDEVICE;
  if (mean) *mean = h.mu;
  if (cscale) *cscale = h.cscale;
  if (scale) *scale = h.scale;
  if (chi0) *chi0 = h.chi0;
  return PSR_OK;
}

int psr_run_batched(psr_ctx* ctx, int njobs, const psr_job* jobs, hipStream_t stream) {
  if (!ctx || njobs < 0 || (njobs > 0 && !jobs)) return PSR_EINVAL;
  for (int i = 0; i < njobs; ++i) {
    const psr_job& j = jobs[i];
    if (j.stages != PSR_JOB_FORWARD && j.stages != PSR_JOB_BACKWARD) return PSR_EINVAL;
    const bool bwd_only = j.stages == PSR_JOB_BACKWARD;
    if ((!bwd_only && (!j.points || !j.normals)) || (bwd_only && !j.dchi)) return PSR_EINVAL;
    if (!j.chi || !j.saved || !j.workspace) return PSR_EINVAL;
    if (!valid_res(j.res) || !valid_P(j.npoints) || !(j.sigma >= 0.0f) || !std::isfinite(j.sigma))
      return PSR_EINVAL;
    if (j.workspace_bytes < psr::ws_layout(j.res, j.npoints).total) return PSR_EINVAL;
    if (!aligned(j.saved, 256) || !aligned(j.workspace, 256) || !aligned(j.chi, 16)) return PSR_EINVAL;
    if (j.dchi && !aligned(j.dchi, 16)) return PSR_EINVAL;
  }
  DeviceGuard g(ctx->device);
  psr::Exec x = make_exec(ctx, stream);
  // group by resolution: one launch per stage and resolution (chunks of
  // psr::kMaxJobs jobs); the forwards of every group, then the backwards
  std::vector<psr::JobArg> fw, bw;
  for (int res = PSR_MIN_RES; res <= PSR_MAX_RES; res *= 2) {
    fw.clear();
    bw.clear();
    for (int i = 0; i < njobs; ++i) {
      const psr_job& j = jobs[i];
      if (j.res != res) continue;
      psr::JobArg a = make_job(j.points, j.normals, j.npoints, j.sigma, j.chi, j.saved, j.workspace);
      if (j.stages == PSR_JOB_FORWARD) fw.push_back(a);
      if (j.dchi) {
        a.dchi = j.dchi;
        a.dpts = j.dpoints;
        a.dnrm = j.dnormals;
        if (int rc = point_source_table(ctx, res, j.sigma, stream, &a.ktab)) return rc;
        bw.push_back(a);
      }
    }
    if (!fw.empty()) {
      if (int rc = psr::run_jobs(x, res, fw.data(), (int)fw.size(), psr::RUN_FORWARD)) return rc;
    }
    if (!bw.empty()) {
      if (int rc = psr::run_jobs(x, res, bw.data(), (int)bw.size(), psr::RUN_BACKWARD)) return rc;
    }
  }
  return PSR_OK;
}

int psr_debug_spectral(psr_ctx* ctx, const float* v, int res, float sigma, float* chi_prime, void* workspace,
                       size_t workspace_bytes, hipStream_t stream) {
  if (!ctx || !v || !chi_prime || !workspace) return PSR_EINVAL;
  if (!valid_res(res) || !(sigma >= 0.0f) || !std::isfinite(sigma)) return PSR_EINVAL;
  if (!aligned(workspace, 256) || !aligned(v, 16)) return PSR_EINVAL;
  if (workspace_bytes < psr::ws_layout(res, 1).total) return PSR_EINVAL;
  DeviceGuard g(ctx->device);
  psr::Exec x = make_exec(ctx, stream);
  psr::JobArg j = make_job(nullptr, nullptr, 1, sigma, nullptr, nullptr, workspace);
  j.aux_in = v;
  j.aux_out = chi_prime;
  return psr::run_debug_spectral(x, res, j);
}

int psr_debug_splat(psr_ctx* ctx, const float* points, const float* normals, int64_t npoints, int res, float* v,
                    void* saved, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!ctx || !points || !normals || !v || !saved || !workspace) return PSR_EINVAL;
  if (!valid_res(res) || !valid_P(npoints)) return PSR_EINVAL;
  if (!aligned(saved, 256) || !aligned(workspace, 256)) return PSR_EINVAL;
  if (workspace_bytes < psr::ws_layout(res, npoints).total) return PSR_EINVAL;
  DeviceGuard g(ctx->device);
  psr::Exec x = make_exec(ctx, stream);
  psr::JobArg j = make_job(points, normals, npoints, 0.0f, nullptr, saved, workspace);
  j.aux_out = v;
  return psr::run_debug_splat(x, res, j);
}

int psr_mc_state_bytes(int res, size_t* bytes) {
  if (!bytes || !valid_res(res)) return PSR_EINVAL;
  *bytes = psr::mc::state_layout(res).total;
  return PSR_OK;
}

int psr_marching_cubes(psr_ctx* ctx, const float* chi, int res, float iso, float* verts, float* normals,
                       int32_t* edges, int64_t vcap, int32_t* tris, int64_t tcap, void* state,
                       hipStream_t stream) {
  if (!ctx || !chi || !state || !valid_res(res) || !std::isfinite(iso) || vcap < 0 || tcap < 0) return PSR_EINVAL;
  if ((vcap > 0 && (!verts || !normals)) || (tcap > 0 && !tris)) return PSR_EINVAL;
  if (!aligned(state, 256) || !aligned(chi, 4)) return PSR_EINVAL;
  DeviceGuard g(ctx->device);
  psr::mc::McOut out{verts, normals, edges, tris, vcap, tcap};
  return psr::mc::run_forward(res, chi, iso, psr::mc::state_view(state, res), out, stream) ? PSR_EDEVICE : PSR_OK;
}

int psr_mc_counts(const void* state, hipStream_t stream, int64_t* nverts, int64_t* ntris, int* status) {
  if (!state) return PSR_EINVAL;
  if (hipStreamSynchronize(stream) != hipSuccess) return PSR_EDEVICE;
  psr::mc::McHeader h;
  if (hipMemcpy(&h, state, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return PSR_EDEVICE;
  if (nverts) *nverts = h.nv;
  if (ntris) *ntris = h.nt;
  if (status) *status = h.status ? PSR_ETOOBIG : PSR_OK;
  return PSR_OK;
}

int psr_marching_cubes_backward(psr_ctx* ctx, const float* chi, int res, float iso, const void* state,
                                const float* normals, const float* dverts, int64_t nverts, float* dchi,
                                hipStream_t stream) {
  if (!ctx || !chi || !state || !dchi || !valid_res(res) || !std::isfinite(iso) || nverts < 0) return PSR_EINVAL;
  if (nverts > 0 && (!normals || !dverts)) return PSR_EINVAL;
  if (!aligned(state, 256)) return PSR_EINVAL;
  DeviceGuard g(ctx->device);
  return psr::mc::run_backward(res, chi, iso, psr::mc::state_view(const_cast<void*>(state), res), normals, dverts,
                               nverts, dchi, stream)
             ? PSR_EDEVICE
             : PSR_OK;
}

int psr_mesh_sample_workspace_bytes(int64_t nfaces, size_t* bytes) {
  if (!bytes || nfaces < 1) return PSR_EINVAL;
  *bytes = psr::opt::sample_layout(nfaces).total;
  return PSR_OK;
}

int psr_mesh_sample(psr_ctx* ctx, const float* verts, const float* vnormals, int64_t nverts, const int32_t* faces,
                    int64_t nfaces, const float* face_weight, const float* u, int64_t nsamples, float* points,
                    float* normals, int32_t* face, float* bary, void* workspace, size_t workspace_bytes,
                    hipStream_t stream) {
  if (!ctx || !verts || nverts < 1 || !faces || nfaces < 1 || nsamples < 0 || !workspace) return PSR_EINVAL;
  if (nsamples > 0 && (!u || !points || !face || !bary || (normals && !vnormals))) return PSR_EINVAL;
  if (workspace_bytes < psr::opt::sample_layout(nfaces).total || !aligned(workspace, 256)) return PSR_EINVAL;
  DeviceGuard g(ctx->device);
  return psr::opt::run_sample(verts, vnormals, faces, nfaces, face_weight, u, nsamples, points, normals, face, bary,
                              workspace, stream)
             ? PSR_EDEVICE
             : PSR_OK;
}

int psr_mesh_sample_backward(psr_ctx* ctx, const int32_t* faces, int64_t nverts, const int32_t* face,
                             const float* bary, const float* dpoints, int64_t nsamples, float* dverts,
                             hipStream_t stream) {
  if (!ctx || !faces || nverts < 1 || nsamples < 0 || !dverts) return PSR_EINVAL;
  if (nsamples > 0 && (!face || !bary || !dpoints)) return PSR_EINVAL;
  DeviceGuard g(ctx->device);
  return psr::opt::run_sample_backward(faces, nverts, face, bary, dpoints, nsamples, dverts, stream) ? PSR_EDEVICE
                                                                                                    : PSR_OK;
}

int psr_chamfer_workspace_bytes(int64_t nx, int64_t ny, size_t* bytes) {
  if (!bytes || nx < 1 || ny < 1) return PSR_EINVAL;
  *bytes = psr::opt::chamfer_ws(nx, ny);
  return PSR_OK;
}

int psr_chamfer(psr_ctx* ctx, const float* x, int64_t nx, const float* y, int64_t ny, int32_t* nn_x, float* d_x,
                int32_t* nn_y, float* d_y, double* loss, void* workspace, size_t workspace_bytes,
                hipStream_t stream) {
  if (!ctx || !x || !y || nx < 1 || ny < 1 || nx >= ((int64_t)1 << 31) || ny >= ((int64_t)1 << 31)) return PSR_EINVAL;
  if (!nn_x || !d_x || !nn_y || !d_y || !workspace) return PSR_EINVAL;
  if (workspace_bytes < psr::opt::chamfer_ws(nx, ny) || !aligned(workspace, 256)) return PSR_EINVAL;
  DeviceGuard g(ctx->device);
  return psr::opt::run_chamfer(x, nx, y, ny, nn_x, d_x, nn_y, d_y, loss, workspace, stream) ? PSR_EDEVICE : PSR_OK;
}

int psr_chamfer_backward(psr_ctx* ctx, const float* x, int64_t nx, const float* y, int64_t ny, const int32_t* nn_x,
                         const int32_t* nn_y, float* grad_x, hipStream_t stream) {
  if (!ctx || !x || !y || nx < 1 || ny < 1 || !nn_x || !nn_y || !grad_x) return PSR_EINVAL;
  DeviceGuard g(ctx->device);
  return psr::opt::run_chamfer_backward(x, nx, y, ny, nn_x, nn_y, grad_x, stream) ? PSR_EDEVICE : PSR_OK;
}

int psr_mesh_components_workspace_bytes(int64_t nverts, int64_t nfaces, size_t* bytes) {
  if (!bytes || nverts < 1 || nfaces < 1) return PSR_EINVAL;
  *bytes = psr::opt::comp_layout(nverts, nfaces).total;
  return PSR_OK;
}

int psr_mesh_components(psr_ctx* ctx, const float* verts, int64_t nverts, const int32_t* faces, int64_t nfaces,
                        int32_t* labels, float* largest, void* workspace, size_t workspace_bytes,
                        hipStream_t stream) {
  if (!ctx || !verts || nverts < 1 || nverts >= ((int64_t)1 << 31) || !faces || nfaces < 1 || !labels) return PSR_EINVAL;
  if (!workspace || workspace_bytes < psr::opt::comp_layout(nverts, nfaces).total || !aligned(workspace, 256))
    return PSR_EINVAL;
  DeviceGuard g(ctx->device);
  // pointer jumping roughly doubles the reach of a label per pass (a mesh of
  // the grids here settles in a few tens of passes); 256 passes at most
  const int rc = psr::opt::run_components(verts, nverts, faces, nfaces, labels, largest, workspace, stream, 256);
  return rc == 0 ? PSR_OK : (rc == -5 ? PSR_ENOTREADY : PSR_EDEVICE);
}

namespace {

// Workspace of psr_opt_step: every buffer of the iteration, 256-byte aligned.
struct OptStepLayout {
  size_t fws, saved, chi, dchi, mcs, verts, vnorm, edges, tris, sws, x, face, bary, cws, nnx, dx, nny, dy, gx, dv, dp,
      dn, total;
  size_t fws_bytes, sws_bytes, cws_bytes;
};

OptStepLayout opt_step_layout(int res, int64_t P, int64_t T, int64_t S, int64_t vcap, int64_t tcap) {
  OptStepLayout L{};
  size_t o = 0;
  auto take = [&](size_t& f, size_t bytes) {
    f = o;
    o += (bytes + 255) & ~(size_t)255;
  };
  const size_t r3 = (size_t)res * res * res;
  size_t mcb = 0;
  psr_mc_state_bytes(res, &mcb);
  L.fws_bytes = psr::ws_layout(res, P).total;
  L.sws_bytes = psr::opt::sample_layout(tcap).total;
  L.cws_bytes = psr::opt::chamfer_ws(S, T);
  take(L.fws, L.fws_bytes);
  take(L.saved, psr::saved_layout(res, P).total);
  take(L.chi, r3 * 4);
  take(L.dchi, r3 * 4);
  take(L.mcs, mcb);
  take(L.verts, (size_t)vcap * 12);
  take(L.vnorm, (size_t)vcap * 12);
  take(L.edges, (size_t)vcap * 4);
  take(L.tris, (size_t)tcap * 12);
  take(L.sws, L.sws_bytes);
  take(L.x, (size_t)S * 12);
  take(L.face, (size_t)S * 4);
  take(L.bary, (size_t)S * 12);
  take(L.cws, L.cws_bytes);
  take(L.nnx, (size_t)S * 4);
  take(L.dx, (size_t)S * 4);
  take(L.nny, (size_t)T * 4);
  take(L.dy, (size_t)T * 4);
  take(L.gx, (size_t)S * 12);
  take(L.dv, (size_t)vcap * 12);
  take(L.dp, (size_t)P * 12);
  take(L.dn, (size_t)P * 12);
  L.total = o;
  return L;
}

bool opt_step_sizes_ok(int res, int64_t P, int64_t T, int64_t S, int64_t vcap, int64_t tcap) {
  constexpr int64_t lim = (int64_t)1 << 31;
  return valid_res(res) && valid_P(P) && T >= 1 && T < lim && S >= 1 && S < lim && vcap >= 1 && vcap < lim &&
         tcap >= 1 && tcap < lim;
}

}  // namespace

int psr_opt_step_workspace_bytes(int res, int64_t npoints, int64_t ntarget, int64_t nsamples, int64_t vcap,
                                 int64_t tcap, size_t* bytes) {
  if (!bytes || !opt_step_sizes_ok(res, npoints, ntarget, nsamples, vcap, tcap)) return PSR_EINVAL;
  *bytes = opt_step_layout(res, npoints, ntarget, nsamples, vcap, tcap).total;
  return PSR_OK;
}

int psr_opt_step(psr_ctx* ctx, float* points, float* normals, int64_t npoints, float* m_points, float* v_points,
                 float* m_normals, float* v_normals, int64_t t, float lr, float beta1, float beta2, float eps,
                 const float* target, int64_t ntarget, const float* u, int64_t nsamples, int res, float sigma,
                 int64_t vcap, int64_t tcap, double* loss, int64_t* mesh_counts, void* workspace,
                 size_t workspace_bytes, hipStream_t stream) {
  if (!ctx || !points || !normals || !m_points || !v_points || !m_normals || !v_normals || !target || !u || !loss ||
      !workspace)
    return PSR_EINVAL;
  if (!opt_step_sizes_ok(res, npoints, ntarget, nsamples, vcap, tcap) || t < 1) return PSR_EINVAL;
  if (!(sigma >= 0.0f) || !std::isfinite(sigma) || !std::isfinite(lr) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
      !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f) || !std::isfinite(eps))
    return PSR_EINVAL;
  if (!aligned(workspace, 256)) return PSR_EINVAL;
  const OptStepLayout L = opt_step_layout(res, npoints, ntarget, nsamples, vcap, tcap);
  if (workspace_bytes < L.total) return PSR_EINVAL;
  char* b = static_cast<char*>(workspace);
  auto f32 = [&](size_t o) { return reinterpret_cast<float*>(b + o); };
  auto i32 = [&](size_t o) { return reinterpret_cast<int32_t*>(b + o); };
  float* chi = f32(L.chi);
  int rc = psr_forward(ctx, points, normals, npoints, res, sigma, chi, b + L.saved, b + L.fws, L.fws_bytes, stream);
  if (rc != PSR_OK) return rc;
  rc = psr_marching_cubes(ctx, chi, res, 0.0f, f32(L.verts), f32(L.vnorm), i32(L.edges), vcap, i32(L.tris), tcap,
                          b + L.mcs, stream);
  if (rc != PSR_OK) return rc;
  int64_t nv = 0, nt = 0;
  int st = PSR_OK;
  rc = psr_mc_counts(b + L.mcs, stream, &nv, &nt, &st);
  if (rc != PSR_OK) return rc;
  if (mesh_counts) {
    mesh_counts[0] = nv;
    mesh_counts[1] = nt;
  }
  if (st != PSR_OK || nv > vcap || nt > tcap) return PSR_ETOOBIG;
  if (nv == 0 || nt == 0) return PSR_EDEGENERATE;
  // forward chain: samples of the mesh, Chamfer loss (main Eq. 5)
  if ((rc = psr_mesh_sample(ctx, f32(L.verts), nullptr, nv, i32(L.tris), nt, nullptr, u, nsamples, f32(L.x), nullptr,
                            i32(L.face), f32(L.bary), b + L.sws, L.sws_bytes, stream)) != PSR_OK)
    return rc;
  if ((rc = psr_chamfer(ctx, f32(L.x), nsamples, target, ntarget, i32(L.nnx), f32(L.dx), i32(L.nny), f32(L.dy), loss,
                        b + L.cws, L.cws_bytes, stream)) != PSR_OK)
    return rc;
  // backward chain: samples -> vertices -> grid (main Eq. 6) -> points and normals
  if ((rc = psr_chamfer_backward(ctx, f32(L.x), nsamples, target, ntarget, i32(L.nnx), i32(L.nny), f32(L.gx),
                                 stream)) != PSR_OK)
    return rc;
  if ((rc = psr_mesh_sample_backward(ctx, i32(L.tris), nv, i32(L.face), f32(L.bary), f32(L.gx), nsamples, f32(L.dv),
                                     stream)) != PSR_OK)
    return rc;
  if ((rc = psr_marching_cubes_backward(ctx, chi, res, 0.0f, b + L.mcs, f32(L.vnorm), f32(L.dv), nv, f32(L.dchi),
                                        stream)) != PSR_OK)
    return rc;
  if ((rc = psr_backward(ctx, npoints, res, sigma, chi, b + L.saved, f32(L.dchi), f32(L.dp), f32(L.dn), b + L.fws,
                         L.fws_bytes, stream)) != PSR_OK)
    return rc;
  DeviceGuard g(ctx->device);
  rc = psr::opt::run_adam(points, m_points, v_points, f32(L.dp), 3 * npoints, t, lr, beta1, beta2, eps, true, stream);
  rc |= psr::opt::run_adam(normals, m_normals, v_normals, f32(L.dn), 3 * npoints, t, lr, beta1, beta2, eps, false,
                           stream);
  return rc ? PSR_EDEVICE : PSR_OK;
}

int psr_mc_case_table(int8_t* ntri, int8_t* edges) {
  if (!ntri && !edges) return PSR_EINVAL;
  psr::mc::case_table(ntri, edges);
  return PSR_OK;
}

int psr_ctx_stage_times(psr_ctx* ctx, double* ms, int64_t* counts, int n) {
  if (!ctx || n < 0) return PSR_EINVAL;
  if (!ctx->timers) return PSR_EINVAL;
  DeviceGuard g(ctx->device);
  ctx->timers->flush();
  for (int i = 0; i < n && i < psr::NUM_STAGES; ++i) {
    if (ms) ms[i] = ctx->timers->ms[i];
    if (counts) counts[i] = ctx->timers->cnt[i];
  }
  return PSR_OK;
}

int psr_ctx_reset_timers(psr_ctx* ctx) {
  if (!ctx || !ctx->timers) return PSR_EINVAL;
  DeviceGuard g(ctx->device);
  ctx->timers->flush();
  for (int i = 0; i < psr::NUM_STAGES; ++i) {
    ctx->timers->ms[i] = 0.0;
    ctx->timers->cnt[i] = 0;
  }
  return PSR_OK;
}

const char* psr_stage_name(int stage) {
  if (stage < 0 || stage >= psr::NUM_STAGES) return "unknown";
  return kStageNames[stage];
}

int psr_num_stages(void) { return psr::NUM_STAGES; }

}  // extern "C"
