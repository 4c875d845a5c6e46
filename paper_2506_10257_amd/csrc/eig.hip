// FP64 eigensolver of the n x n Gram matrix and the singular value
// thresholding weights (paper Sec. II-A, Eq. 4).
//
// For A = X - S + Y/mu (m x n, m pixels, n frames) the thresholded SVD
// D_tau(A) = U max(Lambda - tau, 0) V^T equals A P with
//     P = V diag(w) V^T,   w_i = max(sigma_i - tau, 0) / sigma_i,
// where A^T A = V diag(sigma^2) V^T.  One workgroup per solve:
//
//   0. reduction: add the streaming pass's group partials (Gram, residual,
//      and at the first step sum|X|, sum X^2, non-finite count) in order;
//   1. control: decide whether the solve continues (stopping test of the
//      previous pass, iteration cap, mu and lambda at the first iteration);
//   2. warm start: G~ = V_prev^T G V_prev with the previous eigenvectors,
//      which is nearly diagonal once the iteration settles.  For FP64 solves
//      V_prev is first brought back to orthogonality by one Newton-Schulz
//      step of the polar iteration, V <- V (3I - V^T V) / 2: without it the
//      rounding of the rotations accumulates over hundreds of iterations and
//      the projector drifts away from an orthogonal one at the 1e-12 level,
//      which matters for FP64 data but not for FP32 data;
//   3. cyclic two-sided Jacobi in LDS with the round-robin parallel ordering
//      (each index meets every other once per sweep, n/2 disjoint pairs per
//      round).  G and V are double-buffered: a round reads one copy and
//      writes J^T G J and V J into the other, and the threads that own the
//      next round's pairs compute that round's rotations (and the column
//      table of its J) in the same phase, so a round costs one barrier;
//   4. w from the eigenvalues, P = V diag(w) V^T in the storage precision.
//
// The rotation of a pair is the symmetric 2x2 Schur decomposition with the
// smaller angle (Golub & Van Loan, Matrix Computations, Sec. 8.5), written
// with one division: t = sgn(d) 2 g_pq / (|d| + sqrt(d^2 + 4 g_pq^2)),
// d = g_qq - g_pp, c = 1/sqrt(1 + t^2), s = t c.  A pair is rotated while
// g_pq^2 > eps^2 |g_pp g_qq| (relative off-diagonal test); eps is 1e-15 for
// FP64 solves and 1e-8 for FP32 solves, whose Gram entries carry the data's
// 6e-8 rounding (6x above the off-diagonals left unrotated).
#include <atomic>
#include <type_traits>

#include "common.h"
#include "eig_common.h"
#include "launch.h"

namespace rpca {
namespace {

using namespace eigk;

template <typename T, int NMAX, int NT>
__global__ void __launch_bounds__(NT)
k_eig(const SolveDesc* __restrict__ descs, const int32_t* __restrict__ ids) {
  constexpr int LD = NMAX + 1;
  constexpr int MU = (NMAX * (NMAX + 1) / 2 + NT - 1) / NT;  // upper entries per thread
  constexpr int MF = (NMAX * NMAX + NT - 1) / NT;            // full entries per thread
  __shared__ double G0s[NMAX * LD], G1s[NMAX * LD];  // two copies of G
  __shared__ double V0s[NMAX * LD], V1s[NMAX * LD];  // two copies of V
  __shared__ int cu[2][NMAX];
  __shared__ double2 cab[2][NMAX];
  __shared__ double cd[2][NMAX];
  __shared__ double w[NMAX];
  __shared__ double scal[kScalars];
  __shared__ int s_go;
  __shared__ double s_tau;

  const int tid = threadIdx.x;
  const SolveDesc& d = descs[ids[blockIdx.x]];
  SolveState* st = d.st;
#ifdef RPCA_TRACE
  int64_t tprev = RPCA_NOW();
#define EIG_MARK(i)                               \
  do {                                            \
    if (tid == 0) {                               \
      const int64_t tnow_ = RPCA_NOW();           \
      st->trace[i] += tnow_ - tprev;              \
      tprev = tnow_;                              \
    }                                             \
  } while (0)
#else
#define EIG_MARK(i) \
  do {              \
  } while (0)
#endif

  if (st->done) return;
  const int n = d.n;
  const int nb = d.nb;
  const int kd = st->iter;
  // read now (thread 0 runs the control step), in flight during the reduction
  double pf_nXF2 = 0.0, pf_tau = 0.0;
  if (tid == 0) {
    pf_nXF2 = st->nXF2;
    pf_tau = st->tau;
  }
  const bool warm = kd > 0;
  const int nup = n * (n + 1) / 2;
  const int nfull = n * n;
  const int n4 = (n + 3) & ~3;  // dot products stop here: entries past n are zero

  // Owned entries: upper-triangle (i <= j, column-packed) and full (row-major).
  int ui[MU], uj[MU], fr[MF], fc[MF];
#pragma unroll
  for (int q = 0; q < MU; ++q) {
    const int idx = tid + q * NT;
    int j = 0;
    if (idx < nup) {
      while ((j + 1) * (j + 2) / 2 <= idx) ++j;
    }
    uj[q] = j;
    ui[q] = idx < nup ? idx - j * (j + 1) / 2 : 0;
  }
#pragma unroll
  for (int q = 0; q < MF; ++q) {
    const int idx = tid + q * NT;
    fr[q] = idx < nfull ? idx / n : 0;
    fc[q] = idx < nfull ? idx - fr[q] * n : 0;
  }

  // Previous eigenvectors: issue the loads before the reduction.
  double vpre[MF];
#pragma unroll
  for (int q = 0; q < MF; ++q) {
    vpre[q] = 0.0;
    if (tid + q * NT < nfull) {
      vpre[q] = warm ? d.V[fr[q] * nb + fc[q]] : (fr[q] == fc[q] ? 1.0 : 0.0);
    }
  }

  // Zero the LDS matrices: entries outside n x n stay zero for the whole
  // solve step, so fixed-length dot products need no guards.
  for (int idx = tid; idx < NMAX * LD; idx += NT) {
    G0s[idx] = 0.0;
    G1s[idx] = 0.0;
    V0s[idx] = 0.0;
    V1s[idx] = 0.0;
  }
  if (tid < NMAX) w[tid] = 0.0;
  __syncthreads();

  // 0. Final level of the streaming pass's reduction, Gram straight into LDS.
  {
    const int nblk = gram_blocks((n + 3) >> 2);
    const int nent = kScalars + nblk * 16;
    constexpr int kChunk = 32;  // one batch of loads for up to 32 groups
    for (int idx = tid; idx < nent; idx += NT) {
      double sum = 0.0;
      for (int q0 = 0; q0 < d.groups; q0 += kChunk) {
        const int c = min(kChunk, d.groups - q0);
        double v[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q)
          v[q] = q < c ? d.gpartials[static_cast<size_t>(q0 + q) * d.pstride + idx] : 0.0;
#pragma unroll
        for (int q = 0; q < kChunk; ++q)
          if (q < c) sum += v[q];
      }
      if (idx < kScalars) {
        scal[idx] = sum;
      } else {
        const int g = idx - kScalars;
        const int blk = g >> 4, e = g & 15;
        int bj = 0;
        while ((bj + 1) * (bj + 2) / 2 <= blk) ++bj;
        const int bi = blk - bj * (bj + 1) / 2;
        const int i = 4 * bi + (e >> 2), j = 4 * bj + (e & 3);
        if (i < n && j < n) {
          G0s[i * LD + j] = sum;
          G0s[j * LD + i] = sum;
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < MF; ++q)
    if (tid + q * NT < nfull) V0s[fr[q] * LD + fc[q]] = vpre[q];
  __syncthreads();

  // 1. Control.
  if (tid == 0) {
    double t = 0.0;
    const int go = eigk::control_step(d, st, scal, kd, pf_nXF2, pf_tau, t);
    s_go = go;
    s_tau = t;
  }
  __syncthreads();
  if (!s_go) return;
  EIG_MARK(0);
  const double tau = s_tau;
  int cur = 0;  // which copy (0 or 1) holds the current G and V

  // 2. Warm start.  Each product goes straight into a buffer that is not one
  // of its operands; a barrier separates the products.  FP64 solves first
  // re-orthonormalise V by one Newton-Schulz step (G~ and V1 end in copy 1);
  // for FP32 solves the rotations' rounding drift (about 1e-12 over a
  // thousand steps) stays far below the data's rounding, so G~ = V^T G V is
  // formed directly (G~ and V end in copy 0).
  if (warm) {
    if constexpr (std::is_same<T, double>::value) {
      for (int idx = tid; idx < nup; idx += NT) {  // C = V^T V  -> G1s
        int j = 0;
        while ((j + 1) * (j + 2) / 2 <= idx) ++j;
        const int i = idx - j * (j + 1) / 2;
        const double c = dot4n<NMAX>(n4, [&](int k, double acc) { return fma(V0s[k * LD + i], V0s[k * LD + j], acc); });
        G1s[i * LD + j] = c;
        G1s[j * LD + i] = c;
      }
      __syncthreads();
      for (int idx = tid; idx < nfull; idx += NT) {  // V1 = 1.5 V - 0.5 V C  -> V1s
        const int i = idx / n, j = idx - (idx / n) * n;
        const double vc = dot4n<NMAX>(n4, [&](int k, double acc) { return fma(V0s[i * LD + k], G1s[k * LD + j], acc); });
        V1s[i * LD + j] = fma(-0.5, vc, 1.5 * V0s[i * LD + j]);
      }
      __syncthreads();
      for (int idx = tid; idx < nfull; idx += NT) {  // W = G V1  -> V0s (V is dead)
        const int i = idx / n, j = idx - (idx / n) * n;
        V0s[i * LD + j] = dot4n<NMAX>(n4, [&](int k, double acc) { return fma(G0s[i * LD + k], V1s[k * LD + j], acc); });
      }
      __syncthreads();
      for (int idx = tid; idx < nup; idx += NT) {  // G~ = V1^T W  -> G1s (C is dead)
        int j = 0;
        while ((j + 1) * (j + 2) / 2 <= idx) ++j;
        const int i = idx - j * (j + 1) / 2;
        const double g = dot4n<NMAX>(n4, [&](int k, double acc) { return fma(V1s[k * LD + i], V0s[k * LD + j], acc); });
        G1s[i * LD + j] = g;
        G1s[j * LD + i] = g;
      }
      cur = 1;
    } else {
      for (int idx = tid; idx < nfull; idx += NT) {  // W = G V  -> G1s
        const int i = idx / n, j = idx - (idx / n) * n;
        G1s[i * LD + j] = dot4n<NMAX>(n4, [&](int k, double acc) { return fma(G0s[i * LD + k], V0s[k * LD + j], acc); });
      }
      __syncthreads();
      for (int idx = tid; idx < nup; idx += NT) {  // G~ = V^T W  -> G0s (G is dead)
        int j = 0;
        while ((j + 1) * (j + 2) / 2 <= idx) ++j;
        const int i = idx - j * (j + 1) / 2;
        const double g = dot4n<NMAX>(n4, [&](int k, double acc) { return fma(V0s[k * LD + i], G1s[k * LD + j], acc); });
        G0s[i * LD + j] = g;
        G0s[j * LD + i] = g;
      }
      cur = 0;
    }
    __syncthreads();
  }
  EIG_MARK(1);

  // 3. Jacobi sweeps.
  const int N2 = n + (n & 1);
  const int M = N2 - 1;
  const int NP = N2 / 2;
  int sweeps = 0;
  // One round: read copy SRC and the round's column table, write J^T G J and
  // V J into the other copy; the last wavefront builds the next round's
  // rotations and column table.
  auto round = [&](auto src_tag, int r) {
    constexpr int SRC = decltype(src_tag)::value;
    const double* Gc = SRC ? G1s : G0s;
    double* Gn = SRC ? G0s : G1s;
    const double* Vc = SRC ? V1s : V0s;
    double* Vn = SRC ? V0s : V1s;
    const int rb = r & 1;
    const int* tu_ = cu[rb];
    const double2* tab = cab[rb];
    const double* td = cd[rb];
#pragma unroll
    for (int q = 0; q < MU; ++q) {
      if (tid + q * NT < nup) {  // slots past n(n+1)/2 are skipped by whole waves
        const double v = rotated_entry<LD>(ui[q], uj[q], Gc, tu_, tab, td);
        Gn[ui[q] * LD + uj[q]] = v;
        Gn[uj[q] * LD + ui[q]] = v;
      }
    }
#pragma unroll
    for (int q = 0; q < MF; ++q) {
      if (tid + q * NT < nfull) {
        const int j = fc[q], i = fr[q];
        const int pj = tu_[j];
        const double2 abj = tab[j];
        Vn[i * LD + j] = fma(abj.x, Vc[i * LD + (pj & 0xff)], abj.y * Vc[i * LD + ((pj >> 8) & 0xff)]);
      }
    }
    const int kp = tid - (NT - 64);
    if (r + 1 < M && kp >= 0 && kp < NP) {
      int p, q;
      pair_indices(r + 1, kp, N2, p, q);
      double c = 1.0, s = 0.0, dt = 0.0;
      if (q < n) {
        const double gpp = rotated_entry<LD>(p, p, Gc, tu_, tab, td);
        const double gqq = rotated_entry<LD>(q, q, Gc, tu_, tab, td);
        const double gpq = rotated_entry<LD>(p, q, Gc, tu_, tab, td);
        make_rotation<T>(gpp, gqq, gpq, c, s, dt);
      }
      set_pair_columns(p, q, n, c, s, dt, cu[rb ^ 1], cab[rb ^ 1], cd[rb ^ 1]);
    }
    __syncthreads();
  };
  for (; sweeps < kMaxSweeps && n > 1; ++sweeps) {
    // Convergence test of the current G, and the rotations of round 0.
    const double* G = cur ? G1s : G0s;
    int need = 0;
#pragma unroll
    for (int q = 0; q < MU; ++q) {
      if (tid + q * NT < nup && ui[q] < uj[q]) {
        const int i = ui[q], j = uj[q];
        if (off_diag_large<T>(G[i * LD + j], G[i * LD + i], G[j * LD + j])) need = 1;
      }
    }
    if (tid < NP) {
      int p, q;
      pair_indices(0, tid, N2, p, q);
      double c = 1.0, s = 0.0, dt = 0.0;
      if (q < n) make_rotation<T>(G[p * LD + p], G[q * LD + q], G[p * LD + q], c, s, dt);
      set_pair_columns(p, q, n, c, s, dt, cu[0], cab[0], cd[0]);
    }
    if (!__syncthreads_or(need)) break;
    for (int r = 0; r < M; ++r) {
      if (cur) round(std::integral_constant<int, 1>{}, r);
      else round(std::integral_constant<int, 0>{}, r);
      cur ^= 1;
    }
  }
  EIG_MARK(2);

  // 4. SVT weights and the projector P = V diag(w) V^T (exactly symmetric).
  const double* Gf = cur ? G1s : G0s;
  const double* Vf = cur ? V1s : V0s;
  if (tid < n) {
    const double sg = sqrt(fmax(Gf[tid * LD + tid], 0.0));
    w[tid] = sg > tau ? (sg - tau) / sg : 0.0;
  }
  __syncthreads();
  const gptr<T> Pd = as_global<T>(d.P);
  const int nbup = nb * (nb + 1) / 2;
  for (int idx = tid; idx < nbup; idx += NT) {
    int j = 0;
    while ((j + 1) * (j + 2) / 2 <= idx) ++j;
    const int i = idx - j * (j + 1) / 2;
    double s = 0.0;
    if (j < n) {
      s = dot4n<NMAX>(n4, [&](int k, double acc) { return fma(Vf[i * LD + k] * w[k], Vf[j * LD + k], acc); });
    }
    Pd[i * nb + j] = static_cast<T>(s);
    Pd[j * nb + i] = static_cast<T>(s);
  }
#pragma unroll
  for (int q = 0; q < MF; ++q)
    if (tid + q * NT < nfull) d.V[fr[q] * nb + fc[q]] = Vf[fr[q] * LD + fc[q]];
  EIG_MARK(3);
  if (tid == 0) {
    int rank = 0;
    for (int k = 0; k < n; ++k) rank += w[k] != 0.0 ? 1 : 0;
    st->rank = rank;
    st->sweeps = sweeps;
    st->sweeps_total += sweeps;
    st->iter = kd + 1;
  }
#undef EIG_MARK
}

}  // namespace

int eig_class(int n) {
  if (n <= kEigMaxN) return n <= 16 ? 16 : (n <= 32 ? 32 : 64);
  return n <= kEigWideMaxN ? kEigWideMaxN : (n <= kEigHugeMaxN ? kEigHugeMaxN : 0);
}

namespace {
// Threads per eigensolve workgroup, per [dtype][class 16/32/64].  Defaults
// from timing on MI355X: a round's work is spread over more waves as n grows.
std::atomic<int> g_eig_nt[2][3] = {{{256}, {512}, {1024}}, {{256}, {512}, {1024}}};
int cls_index(int ncls) { return ncls == 16 ? 0 : (ncls == 32 ? 1 : (ncls == 64 ? 2 : -1)); }
}  // namespace

bool eig_threads_valid(int ncls, int nt) {
  if (cls_index(ncls) < 0) return false;
  return nt == 256 || nt == 512 || (nt == 1024 && ncls >= 32);
}

int eig_threads(int dtype, int ncls) {
  const int c = cls_index(ncls);
  return c < 0 ? 0 : g_eig_nt[dtype == 0 ? 0 : 1][c].load(std::memory_order_relaxed);
}

bool set_eig_threads(int dtype, int ncls, int nt) {
  if (!eig_threads_valid(ncls, nt)) return false;
  g_eig_nt[dtype == 0 ? 0 : 1][cls_index(ncls)].store(nt, std::memory_order_relaxed);
  return true;
}

hipError_t launch_eig(int dtype, int ncls, int grid, hipStream_t stream, const SolveDesc* descs,
                      const int32_t* ids) {
  if (grid <= 0) return hipSuccess;
  const int nt = eig_threads(dtype, ncls);
  const dim3 g(grid), b(nt);
#define RPCA_EIG_CASE(N, NT)                                                  \
  if (ncls == N && nt == NT) {                                                \
    if (dtype == 0)                                                           \
      RPCA_LAUNCH((k_eig<double, N, NT>), g, b, 0, stream, descs, ids); \
    else                                                                      \
      RPCA_LAUNCH((k_eig<float, N, NT>), g, b, 0, stream, descs, ids);  \
    return hipGetLastError();                                                 \
  }
  RPCA_EIG_CASE(16, 256)
  RPCA_EIG_CASE(16, 512)
  RPCA_EIG_CASE(32, 256)
  RPCA_EIG_CASE(32, 512)
  RPCA_EIG_CASE(32, 1024)
  RPCA_EIG_CASE(64, 256)
  RPCA_EIG_CASE(64, 512)
  RPCA_EIG_CASE(64, 1024)
#undef RPCA_EIG_CASE
  return hipErrorInvalidValue;
}

}  // namespace rpca
