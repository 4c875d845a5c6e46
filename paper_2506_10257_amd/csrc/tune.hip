// Autotuner of the launch choices (rpca_autotune* in include/rpca.h).
//
// For each tunable it runs short solves of a synthetic window through the
// library's own solve path with kernel timing on, and keeps the fastest
// variant:
//   * eigensolver workgroup size (256/512/1024 threads) per eigensolver
//     class, timed on an n = class window (the variants compute the same
//     arithmetic, so only time differs);
//   * streaming kernel (thread-per-row register kernel or the MFMA tile
//     kernel) per FP32 register frame class, timed on a window of `rows`
//     pixel rows;
//   * the tile shape of the tile kernel (pixel rows per workgroup) for every
//     tile class that runs it after the step above, timed the same way.
// The synthetic window is a hash-noise matrix with a rank-one background,
// written by a device kernel; timing does not depend on its values except
// through the number of Jacobi sweeps, which is the same for every variant
// of a class.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "rpca.h"
#include "common.h"
#include "engine.h"
#include "launch.h"

namespace rpca {
namespace {

__device__ inline uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

template <typename T>
__global__ void k_fill(T* X, int64_t m, int n) {
  const int64_t total = m * static_cast<int64_t>(n);
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t p = i % m, t = i / m;
    const float u = (mix32(static_cast<uint32_t>(i) * 2654435761u + 12345u) >> 8) * (1.0f / 16777216.0f);
    const float bg = 1.0f + 0.05f * static_cast<float>((p * 7 + t * 3) % 11);
    X[i] = static_cast<T>(bg + 0.5f * u);
  }
}

struct Bufs {
  void* M = nullptr;
  void* L = nullptr;
  void* S = nullptr;
};

int alloc_window(Bufs& b, int64_t m, int n, int dtype, hipStream_t s) {
  const size_t bytes = static_cast<size_t>(m) * n * (dtype == RPCA_F32 ? 4 : 8);
  if (hipMalloc(&b.M, bytes) != hipSuccess || hipMalloc(&b.L, bytes) != hipSuccess ||
      hipMalloc(&b.S, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return RPCA_ERR_NOMEM;
  }
  if (dtype == RPCA_F32)
    hipLaunchKernelGGL(k_fill<float>, dim3(1024), dim3(256), 0, s, static_cast<float*>(b.M), m, n);
  else
    hipLaunchKernelGGL(k_fill<double>, dim3(1024), dim3(256), 0, s, static_cast<double*>(b.M), m, n);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return RPCA_ERR_DEVICE;
  return RPCA_OK;
}

void free_window(Bufs& b) {
  if (b.M) (void)hipFree(b.M);
  if (b.L) (void)hipFree(b.L);
  if (b.S) (void)hipFree(b.S);
  b = Bufs{};
}

// Mean eigensolve and update-launch times (ms) of `iters` iterations.
int time_solve(const Bufs& b, int64_t m, int n, int dtype, int iters, hipStream_t s, double& eig_ms,
               double& upd_ms) {
  rpca_problem p;
  std::memset(&p, 0, sizeof(p));
  p.M = b.M;
  p.L = b.L;
  p.S = b.S;
  p.m = m;
  p.n = n;
  p.lambda = -1.0;
  p.mu = -1.0;
  p.tol = 0.0;
  p.maxit = 3;
  int rc = rpca_solve_ex(&p, dtype, RPCA_GRAM_DEFAULT, s);  // warm-up
  if (rc < 0) return rc;
  rpca_profile pr;
  (void)rpca_profile_read(&pr, 1);
  rpca_profile_enable(1);
  p.maxit = iters;
  rc = rpca_solve_ex(&p, dtype, RPCA_GRAM_DEFAULT, s);
  rpca_profile_enable(0);
  (void)rpca_profile_read(&pr, 1);
  if (rc < 0) return rc;
  eig_ms = pr.eig_launches ? pr.eig_ms / static_cast<double>(pr.eig_launches) : 0.0;
  upd_ms = pr.update_launches ? pr.update_ms / static_cast<double>(pr.update_launches) : 0.0;
  return RPCA_OK;
}

constexpr int kTuneEigRows = 16384;
constexpr int kTuneIters = 12;

}  // namespace
}  // namespace rpca

using namespace rpca;

extern "C" {

int rpca_autotune(int32_t dtype, int64_t rows, void* stream) {
  if (dtype != RPCA_F32 && dtype != RPCA_F64) return RPCA_ERR_ARG;
  if (rows < 256) return RPCA_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = RPCA_OK;

  // 1. eigensolver workgroup size per class
  for (int cls : {16, 32, 64}) {
    Bufs b;
    rc = alloc_window(b, kTuneEigRows, cls, dtype, s);
    if (rc != RPCA_OK) {
      free_window(b);
      return rc;
    }
    const int old = rpca_tune_get(RPCA_KNOB_EIG_THREADS, dtype, cls);
    int best = old;
    double best_ms = 1e30;
    for (int nt : {256, 512, 1024}) {
      if (rpca_tune_set(RPCA_KNOB_EIG_THREADS, dtype, cls, nt) != RPCA_OK) continue;
      double eig_ms = 0, upd_ms = 0;
      rc = time_solve(b, kTuneEigRows, cls, dtype, kTuneIters, s, eig_ms, upd_ms);
      if (rc < 0) break;
      if (eig_ms < best_ms) {
        best_ms = eig_ms;
        best = nt;
      }
    }
    (void)rpca_tune_set(RPCA_KNOB_EIG_THREADS, dtype, cls, rc < 0 ? old : best);
    free_window(b);
    if (rc < 0) return rc;
  }

  // 2. streaming kernel per FP32 register class
  if (dtype == RPCA_F32) {
    for (int cls : kClassesF32) {
      if (cls < 16) continue;  // the tile kernel's smallest class is 16 frames
      Bufs b;
      rc = alloc_window(b, rows, cls, dtype, s);
      if (rc != RPCA_OK) {
        free_window(b);
        return rc;
      }
      const int old = rpca_tune_get(RPCA_KNOB_STREAM_KERNEL, dtype, cls);
      double t[2] = {1e30, 1e30};
      for (int v = 0; v < 2 && rc >= 0; ++v) {
        (void)rpca_tune_set(RPCA_KNOB_STREAM_KERNEL, dtype, cls, v);
        double eig_ms = 0, upd_ms = 0;
        rc = time_solve(b, rows, cls, dtype, kTuneIters, s, eig_ms, upd_ms);
        if (rc >= 0) t[v] = upd_ms;
      }
      (void)rpca_tune_set(RPCA_KNOB_STREAM_KERNEL, dtype, cls, rc < 0 ? old : (t[1] < t[0] ? 1 : 0));
      free_window(b);
      if (rc < 0) return rc;
    }
  }

  // 3. rows per workgroup of the tile kernel, per tile class that runs it:
  // every class above 64 frames, and the classes of the register frame
  // counts whose kernel choice is now the tile kernel (timed with that frame
  // count, so the solve takes the tile kernel)
  if (dtype == RPCA_F32) {
    for (int nb = 16; nb <= kEigHugeMaxN; nb += 16) {
      int n = 0;
      if (nb > kEigMaxN) {
        n = nb;
      } else {
        for (int c : kClassesF32)
          if ((c + 15) / 16 * 16 == nb && rpca_tune_get(RPCA_KNOB_STREAM_KERNEL, dtype, c) == 1) n = c;
      }
      if (n == 0) continue;
      Bufs b;
      rc = alloc_window(b, rows, n, dtype, s);
      if (rc != RPCA_OK) {
        free_window(b);
        return rc;
      }
      const int old = rpca_tune_get(RPCA_KNOB_TILE_ROWS, dtype, nb);
      int best = old;
      double best_ms = 1e30;
      for (int tr : {256, 512, 1024, 2048, 4096}) {
        if (rpca_tune_set(RPCA_KNOB_TILE_ROWS, dtype, nb, tr) != RPCA_OK) continue;
        double eig_ms = 0, upd_ms = 0;
        rc = time_solve(b, rows, n, dtype, kTuneIters, s, eig_ms, upd_ms);
        if (rc < 0) break;
        if (upd_ms < best_ms) {
          best_ms = upd_ms;
          best = tr;
        }
      }
      (void)rpca_tune_set(RPCA_KNOB_TILE_ROWS, dtype, nb, rc < 0 ? old : best);
      free_window(b);
      if (rc < 0) return rc;
    }
  }
  // 4. tiles per workgroup of the register kernel, per register class still
  // on it (FP64: every class), timed on a `rows` x cls window
  {
    const int* cls_list = dtype == RPCA_F32 ? kClassesF32 : kClassesF64;
    const int ncls = dtype == RPCA_F32 ? static_cast<int>(sizeof(kClassesF32) / sizeof(int))
                                       : static_cast<int>(sizeof(kClassesF64) / sizeof(int));
    for (int ci = 0; ci < ncls; ++ci) {
      const int cls = cls_list[ci];
      if (dtype == RPCA_F32 && rpca_tune_get(RPCA_KNOB_STREAM_KERNEL, dtype, cls) != 0) continue;
      Bufs b;
      rc = alloc_window(b, rows, cls, dtype, s);
      if (rc != RPCA_OK) {
        free_window(b);
        return rc;
      }
      const int old = rpca_tune_get(RPCA_KNOB_REG_TILES, dtype, cls);
      int best = old;
      double best_ms = 1e30;
      for (int tw : {1, 2, 4}) {
        if (rpca_tune_set(RPCA_KNOB_REG_TILES, dtype, cls, tw) != RPCA_OK) continue;
        double eig_ms = 0, upd_ms = 0;
        rc = time_solve(b, rows, cls, dtype, kTuneIters, s, eig_ms, upd_ms);
        if (rc < 0) break;
        if (upd_ms < best_ms) {
          best_ms = upd_ms;
          best = tw;
        }
      }
      (void)rpca_tune_set(RPCA_KNOB_REG_TILES, dtype, cls, rc < 0 ? old : best);
      free_window(b);
      if (rc < 0) return rc;
    }
  }
  return RPCA_OK;
}

int rpca_autotune_save(const char* path) {
  if (!path) return RPCA_ERR_ARG;
  FILE* f = std::fopen(path, "w");
  if (!f) return RPCA_ERR_ARG;
  std::fprintf(f, "# rpca_mi355x tuning choices: knob dtype class value\n");
  for (int dt : {RPCA_F64, RPCA_F32})
    for (int cls : {16, 32, 64})
      std::fprintf(f, "%d %d %d %d\n", RPCA_KNOB_EIG_THREADS, dt, cls,
                   rpca_tune_get(RPCA_KNOB_EIG_THREADS, dt, cls));
  for (int cls : kClassesF32)
    std::fprintf(f, "%d %d %d %d\n", RPCA_KNOB_STREAM_KERNEL, RPCA_F32, cls,
                 rpca_tune_get(RPCA_KNOB_STREAM_KERNEL, RPCA_F32, cls));
  for (int nb = 16; nb <= kEigHugeMaxN; nb += 16)
    std::fprintf(f, "%d %d %d %d\n", RPCA_KNOB_TILE_ROWS, RPCA_F32, nb,
                 rpca_tune_get(RPCA_KNOB_TILE_ROWS, RPCA_F32, nb));
  for (int cls : kClassesF32)
    std::fprintf(f, "%d %d %d %d\n", RPCA_KNOB_REG_TILES, RPCA_F32, cls,
                 rpca_tune_get(RPCA_KNOB_REG_TILES, RPCA_F32, cls));
  for (int cls : kClassesF64)
    std::fprintf(f, "%d %d %d %d\n", RPCA_KNOB_REG_TILES, RPCA_F64, cls,
                 rpca_tune_get(RPCA_KNOB_REG_TILES, RPCA_F64, cls));
  const int ok = std::fclose(f) == 0;
  return ok ? RPCA_OK : RPCA_ERR_ARG;
}

int rpca_autotune_load(const char* path) {
  if (!path) return RPCA_ERR_ARG;
  FILE* f = std::fopen(path, "r");
  if (!f) return RPCA_ERR_ARG;
  char line[256];
  int rc = RPCA_OK;
  while (std::fgets(line, sizeof(line), f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    int knob, dt, cls, value;
    if (std::sscanf(line, "%d %d %d %d", &knob, &dt, &cls, &value) != 4 ||
        rpca_tune_set(knob, dt, cls, value) != RPCA_OK)
      rc = RPCA_ERR_ARG;  // keep going: every valid line is applied
  }
  std::fclose(f);
  return rc;
}

}  // extern "C"
