// Device-side data structures shared by the kernels and the host runtime.
//
// One "solve" is one RPCA problem (paper Sec. II-A).  Everything a solve needs
// on the device is described by a SolveDesc that lives in device memory; the
// kernels take an array of them, so one launch can serve many solves.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpca {

constexpr int kThreads = 256;      // threads per streaming workgroup
constexpr int kTile = 256;         // pixel rows per tile: one row per thread
constexpr int kGroup = 32;         // partial slots per first-level reduction group
constexpr int kEigMaxN = 64;       // frame count handled by the double-buffered eigensolver
constexpr int kEigWideMaxN = 112;  // frame count handled by the in-place eigensolver (V in LDS)
constexpr int kEigHugeMaxN = 144;  // ... and by its variant with V in global memory
constexpr int kF64MaxN = 128;      // largest frame count of FP64 solves (tile kernel classes to 128)
constexpr int kEigWideThreads = 1024;
constexpr int kWideRows = 64;      // pixel rows per tile of the MFMA streaming kernel
constexpr int kScalars = 4;        // scalar slots at the head of each partial

// Status codes (mirrors include/rpca.h).
constexpr int kOk = 0;
constexpr int kNotConverged = 1;
constexpr int kErrNonfinite = -4;

// Per-solve iteration state, written only by device code once the solve runs.
struct SolveState {
  double mu, imu, lam, gamma, tau;  // penalty, 1/mu, sparsity weight, lam/mu, 1/mu
  double nX1;                       // sum |X_ij|
  double nXF2;                      // sum X_ij^2
  double r2;                        // ||X - L_k - S_k||_F^2 of the last pass
  double resid;                     // ||X - L - S||_F / ||X||_F at the last check
  int32_t iter;                     // passes started (k of the current iterate)
  int32_t done;                     // 1 once finished (converged, capped or error)
  int32_t status;                   // final status (valid once done)
  int32_t rank;                     // #singular values above tau in the last SVT
  int32_t nonfinite;                // non-finite entries seen by the init pass
  int32_t sweeps;                   // Jacobi sweeps of the last eigensolve
  int32_t sweeps_total;             // over the whole solve
  int32_t warm_stage;               // given start: 0 norms pending, 1 Gram of A_1 pending, 2 running
  int64_t trace[8];                 // phase times of the eigensolve (trace builds only)
};

struct SolveDesc {
  const void* X;          // m x n, column-major, ld = m
  void* S[2];             // ping-pong S iterates (m x n)
  void* Y[2];             // ping-pong Y iterates (m x n)
  void* Lout;             // caller's L
  void* Sout;             // caller's S
  void* Yout;             // caller's Y (optional, else null)
  const void* S0;         // caller's starting S (optional; null = zero)
  const void* Y0;         // caller's starting Y (optional; null = zero)
  double* partials;       // slots x pstride
  double* gpartials;      // groups x pstride
  void* P;                // nb x nb thresholding projector, storage precision
  double* V;              // nb x nb eigenvectors of the last eigensolve
  double* escratch;       // class^2 doubles (112^2 or 144^2) for the wide eigensolver (else null)
  SolveState* st;
  int64_t* wgtrace;       // per-slot timestamps (trace builds only, else null)
  int64_t m;
  int32_t n, nb;          // frames and the compiled frame class (n <= nb)
  int32_t tiles, tps;     // ceil(m / kTile); tiles per slot (always 1)
  int32_t slots, groups;  // partial slots (= tiles); ceil(slots / kGroup)
  int32_t pstride;        // doubles per partial slot
  int32_t maxit;
  int32_t warm;           // 1 when the solve starts from a given S0 / Y0
  double lam_in, mu_in, tol;
};

// Trace builds (-DRPCA_TRACE) record wall-clock timestamps (100 MHz counter)
// at phase boundaries; normal builds compile the hooks away.
#ifdef RPCA_TRACE
#define RPCA_NOW() static_cast<int64_t>(wall_clock64())
#else
#define RPCA_NOW() int64_t(0)
#endif

// Address-space views of device pointers held in descriptors.  A pointer
// loaded from memory is generic to the compiler; naming the global space lets
// it use global (not flat) loads and stores, and naming the constant space for
// data that a launch only reads (the projector, written by the previous
// launch) lets uniform reads become scalar loads.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

template <typename T>
__device__ inline gptr<T> as_global(void* p) {
  return (gptr<T>)(p);
}
template <typename T>
__device__ inline gptr<const T> as_global(const void* p) {
  return (gptr<const T>)(p);
}
template <typename T>
__device__ inline cptr<T> as_const(const void* p) {
  return (cptr<T>)(p);
}

struct WorkItem {
  int32_t solve;   // index into the SolveDesc array of the launch
  int32_t slot;    // which tile: rows [slot * kTile, (slot + 1) * kTile)
};

struct GroupItem {
  int32_t solve;   // index into the SolveDesc array of the launch
  int32_t group;   // slots [group * kGroup, min((group + 1) * kGroup, slots))
};

// Gram blocks: 4 x 4 blocks (bi <= bj) of the n x n Gram, packed by column
// of blocks, so the first b(b+1)/2 blocks cover frames [0, 4b).
__host__ __device__ inline constexpr int gram_blocks(int nb4) { return nb4 * (nb4 + 1) / 2; }
__host__ __device__ inline constexpr int pstride_for(int nb) {
  return kScalars + gram_blocks((nb + 3) / 4) * 16;
}

}  // namespace rpca
