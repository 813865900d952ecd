// Tile-shape autotuner for the grouped (batched) products.
//
// Dimensions are bucketed (N <= 256, <= 1024, <= 4096, larger); for each
// bucket and precision the table holds the tile variant of the grouped
// kernel (1: 128 x 128 tiles / 8 waves, 2: 64 x 64 tiles / 4 waves).
// tc_autotune times both variants on an N x N x N complex product at each
// bucket's representative size with hipEvents and keeps the faster one.  If
// the environment variable TC_AUTOTUNE_CACHE names a file, the table is read
// from it on first use and written to it after tuning (a small JSON object).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "common.h"
#include "gemm_mfma.h"

namespace tcm {
namespace {

constexpr int NB = 4;
const int64_t kBucketMax[NB] = {256, 1024, 4096, int64_t(1) << 40};
const int64_t kBucketRep[NB] = {256, 1024, 4096, 7168};

std::mutex g_mu;
bool g_loaded = false;
// defaults from timing on gfx950: FP32 small products prefer 64 x 64 tiles
int g_table[2][NB] = {{2, 2, 1, 1},    // FP32
                      {2, 2, 2, 2}};   // FP64

int bucket_of(int64_t N) {
  for (int b = 0; b < NB; ++b)
    if (N <= kBucketMax[b]) return b;
  return NB - 1;
}

const char* cache_path() { return getenv("TC_AUTOTUNE_CACHE"); }

void load_cache_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* p = cache_path();
  if (!p) return;
  std::ifstream f(p);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  // {"f32": [v0, v1, v2, v3], "f64": [v0, v1, v2, v3]}
  for (int prec = 0; prec < 2; ++prec) {
    const char* key = prec == 0 ? "\"f32\"" : "\"f64\"";
    const size_t k = s.find(key);
    if (k == std::string::npos) continue;
    const size_t lb = s.find('[', k);
    if (lb == std::string::npos) continue;
    int vals[NB];
    int got = 0;
    const char* c = s.c_str() + lb + 1;
    while (got < NB && *c) {
      char* end = nullptr;
      const long v = strtol(c, &end, 10);
      if (end == c) { ++c; continue; }
      vals[got++] = int(v);
      c = end;
    }
    if (got == NB) {
      bool ok = true;
      for (int b = 0; b < NB; ++b) ok = ok && (vals[b] == 1 || vals[b] == 2);
      if (ok) for (int b = 0; b < NB; ++b) g_table[prec][b] = vals[b];
    }
  }
}

void save_cache_locked() {
  const char* p = cache_path();
  if (!p) return;
  std::ofstream f(p);
  if (!f) return;
  f << "{\"f32\": [" << g_table[0][0] << ", " << g_table[0][1] << ", " << g_table[0][2] << ", "
    << g_table[0][3] << "], \"f64\": [" << g_table[1][0] << ", " << g_table[1][1] << ", "
    << g_table[1][2] << ", " << g_table[1][3] << "]}\n";
}

}  // namespace

int tile_variant_for(int64_t N, bool f64) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_cache_locked();
  return g_table[f64 ? 1 : 0][bucket_of(N)];
}

}  // namespace tcm

using namespace tcm;

extern "C" {

int tc_autotune_workspace_size(int32_t gemm_mode, int64_t max_N, size_t* bytes) {
  clear_error();
  TC_CHECK_ARG(bytes != nullptr, "bytes is NULL");
  TC_CHECK_ARG(gemm_mode == TC_GEMM_F64 || gemm_mode == TC_GEMM_F32, "autotune covers F64 and F32");
  TC_CHECK_ARG(max_N >= 1 && max_N <= (int64_t(1) << 20), "max_N out of range");
  const size_t eb = gemm_mode == TC_GEMM_F64 ? 16 : 8;
  Arena ar(nullptr, 0);
  for (int k = 0; k < 3; ++k) ar.take(size_t(max_N) * size_t(max_N) * eb);
  ar.take(grouped_bytes(1));
  *bytes = ar.used;
  return TC_OK;
}

int tc_autotune(int32_t gemm_mode, int64_t max_N, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  size_t need = 0;
  TC_RETURN_IF(tc_autotune_workspace_size(gemm_mode, max_N, &need));
  TC_CHECK_ARG(ws != nullptr, "workspace is NULL");
  if (ws_bytes < need) { set_error("workspace too small for tc_autotune"); return TC_ERR_WORKSPACE; }
  const bool f64 = gemm_mode == TC_GEMM_F64;
  const size_t eb = f64 ? 16 : 8;
  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);
  void* A = ar.take(size_t(max_N) * size_t(max_N) * eb);
  void* B = ar.take(size_t(max_N) * size_t(max_N) * eb);
  void* C = ar.take(size_t(max_N) * size_t(max_N) * eb);
  void* items = ar.take(grouped_bytes(1));
  // finite non-zero operands (bytes 0x3c: 0.0115 in FP32, 1.5e-18 in FP64)
  TC_TRY_HIP(hipMemsetAsync(A, 0x3c, size_t(max_N) * size_t(max_N) * eb, s));
  TC_TRY_HIP(hipMemsetAsync(B, 0x3c, size_t(max_N) * size_t(max_N) * eb, s));
  hipEvent_t e0, e1;
  TC_TRY_HIP(hipEventCreate(&e0));
  TC_TRY_HIP(hipEventCreate(&e1));
  int chosen[NB];
  int rc = TC_OK;
  for (int b = 0; b < NB && rc == TC_OK; ++b) {
    const int64_t N = std::min<int64_t>(kBucketRep[b], max_N);
    float best = INFINITY;
    chosen[b] = 1;
    for (int v = 1; v <= 2 && rc == TC_OK; ++v) {
      GemmDesc d;
      d.M = d.N = d.K = N;
      d.A = A; d.lda = N; d.a_kmaj = false;
      d.B = B; d.ldb = N; d.b_kmaj = true;
      d.C = C; d.ldc = N;
      GroupedProducts g;
      rc = grouped_build({d}, f64, v, items, &g, s);
      if (rc != TC_OK) break;
      rc = grouped_run(g, s);                     // warm-up
      if (rc != TC_OK) break;
      if (hipEventRecord(e0, s) != hipSuccess) { rc = TC_ERR_HIP; break; }
      for (int r = 0; r < 3 && rc == TC_OK; ++r) rc = grouped_run(g, s);
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        rc = TC_ERR_HIP;
        break;
      }
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = TC_ERR_HIP; break; }
      if (ms < best) { best = ms; chosen[b] = v; }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != TC_OK) {
    if (rc == TC_ERR_HIP) set_error("tc_autotune: HIP event failure");
    return rc;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_loaded = true;
  for (int b = 0; b < NB; ++b) g_table[f64 ? 1 : 0][b] = chosen[b];
  save_cache_locked();
  return TC_OK;
}

int tc_autotune_query(int32_t gemm_mode, int64_t N, int32_t* variant) {
  clear_error();
  TC_CHECK_ARG(variant != nullptr, "variant is NULL");
  TC_CHECK_ARG(gemm_mode == TC_GEMM_F64 || gemm_mode == TC_GEMM_F32, "autotune covers F64 and F32");
  TC_CHECK_ARG(N >= 1, "N < 1");
  *variant = tile_variant_for(N, gemm_mode == TC_GEMM_F64);
  return TC_OK;
}

}  // extern "C"
