// A host program that uses the solver only through its C ABI (include/psr.h)
// and the HIP runtime for device memory: one forward solve (main Eqs. 2-4)
// and its backward for a loss gradient G, as a C or C++ caller would run
// them without Python.
//
//   psr_roundtrip IN OUT
//
// IN (little-endian): int64 P, int32 res, float32 sigma, float32 points[P][3],
// float32 normals[P][3], float32 G[res^3].
// OUT: int32 status, float64 mean, cscale, scale, chi0, float32 chi[res^3],
// float32 dpoints[P][3], float32 dnormals[P][3].
// Exit code 0 on success; a failing call prints its name and status text.
#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "psr.h"

namespace {

bool ok_psr(int rc, const char* what) {
  if (rc == PSR_OK) return true;
  std::fprintf(stderr, "%s: %s (%d)\n", what, psr_strerror(rc), rc);
  return false;
}

bool ok_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  std::fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
  return false;
}

template <typename T>
bool read_n(std::FILE* f, T* p, size_t n) {
  return std::fread(p, sizeof(T), n, f) == n;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: %s IN OUT\n", argv[0]);
    return 2;
  }
  std::FILE* fi = std::fopen(argv[1], "rb");
  if (!fi) return 2;
  int64_t P = 0;
  int32_t res = 0;
  float sigma = 0.0f;
  if (!read_n(fi, &P, 1) || !read_n(fi, &res, 1) || !read_n(fi, &sigma, 1) || P < 1 || res < 8 || res > 512)
    return 2;
  const size_t N = (size_t)res * res * res;
  std::vector<float> pts(3 * P), nrm(3 * P), G(N);
  if (!read_n(fi, pts.data(), pts.size()) || !read_n(fi, nrm.data(), nrm.size()) || !read_n(fi, G.data(), N))
    return 2;
  std::fclose(fi);

  psr_ctx* ctx = nullptr;
  if (!ok_psr(psr_ctx_create(&ctx, 0), "psr_ctx_create")) return 1;
  size_t ws_bytes = 0, sv_bytes = 0;
  if (!ok_psr(psr_workspace_bytes(res, P, 1, &ws_bytes), "psr_workspace_bytes") ||
      !ok_psr(psr_saved_bytes(res, P, &sv_bytes), "psr_saved_bytes"))
    return 1;
  float *d_pts, *d_nrm, *d_chi, *d_G, *d_dp, *d_dn;
  void *d_ws, *d_sv;
  hipStream_t stream;
  if (!ok_hip(hipStreamCreate(&stream), "hipStreamCreate") ||
      !ok_hip(hipMalloc(&d_pts, 12 * P), "hipMalloc") || !ok_hip(hipMalloc(&d_nrm, 12 * P), "hipMalloc") ||
      !ok_hip(hipMalloc(&d_dp, 12 * P), "hipMalloc") || !ok_hip(hipMalloc(&d_dn, 12 * P), "hipMalloc") ||
      !ok_hip(hipMalloc(&d_chi, 4 * N), "hipMalloc") || !ok_hip(hipMalloc(&d_G, 4 * N), "hipMalloc") ||
      !ok_hip(hipMalloc(&d_ws, ws_bytes), "hipMalloc") || !ok_hip(hipMalloc(&d_sv, sv_bytes), "hipMalloc"))
    return 1;
  if (!ok_hip(hipMemcpy(d_pts, pts.data(), 12 * P, hipMemcpyHostToDevice), "hipMemcpy") ||
      !ok_hip(hipMemcpy(d_nrm, nrm.data(), 12 * P, hipMemcpyHostToDevice), "hipMemcpy") ||
      !ok_hip(hipMemcpy(d_G, G.data(), 4 * N, hipMemcpyHostToDevice), "hipMemcpy"))
    return 1;

  if (!ok_psr(psr_forward(ctx, d_pts, d_nrm, P, res, sigma, d_chi, d_sv, d_ws, ws_bytes, stream), "psr_forward"))
    return 1;
  int32_t status = 0;
  double sc[4] = {0, 0, 0, 0};
  if (!ok_psr(psr_saved_status(d_sv, stream, &status), "psr_saved_status") ||
      !ok_psr(psr_saved_scalars(d_sv, stream, &sc[0], &sc[1], &sc[2], &sc[3]), "psr_saved_scalars"))
    return 1;
  if (!ok_psr(psr_backward(ctx, P, res, sigma, d_chi, d_sv, d_G, d_dp, d_dn, d_ws, ws_bytes, stream),
              "psr_backward"))
    return 1;
  if (!ok_hip(hipStreamSynchronize(stream), "hipStreamSynchronize")) return 1;

  std::vector<float> chi(N), dp(3 * P), dn(3 * P);
  if (!ok_hip(hipMemcpy(chi.data(), d_chi, 4 * N, hipMemcpyDeviceToHost), "hipMemcpy") ||
      !ok_hip(hipMemcpy(dp.data(), d_dp, 12 * P, hipMemcpyDeviceToHost), "hipMemcpy") ||
      !ok_hip(hipMemcpy(dn.data(), d_dn, 12 * P, hipMemcpyDeviceToHost), "hipMemcpy"))
    return 1;
  std::FILE* fo = std::fopen(argv[2], "wb");
  if (!fo) return 2;
  std::fwrite(&status, 4, 1, fo);
  std::fwrite(sc, 8, 4, fo);
  std::fwrite(chi.data(), 4, N, fo);
  std::fwrite(dp.data(), 4, dp.size(), fo);
  std::fwrite(dn.data(), 4, dn.size(), fo);
  std::fclose(fo);

  for (void* p : {(void*)d_pts, (void*)d_nrm, (void*)d_dp, (void*)d_dn, (void*)d_chi, (void*)d_G, d_ws, d_sv})
    (void)hipFree(p);
  (void)hipStreamDestroy(stream);
  return ok_psr(psr_ctx_destroy(ctx), "psr_ctx_destroy") ? 0 : 1;
}
