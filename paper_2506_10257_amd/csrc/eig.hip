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
//      which is nearly diagonal once the iteration settles.  V_prev is first
//      brought back to orthogonality by one Newton-Schulz step of the polar
//      iteration, V <- V (3I - V^T V) / 2: without it the rounding of the
//      rotations accumulates over hundreds of iterations and the projector
//      drifts away from an orthogonal one;
//   3. cyclic two-sided Jacobi in LDS with the round-robin parallel ordering:
//      each round rotates n/2 disjoint (p, q) pairs at once, so a round is
//      one barrier-separated update of all of G and V;
//   4. w from the eigenvalues, P = V diag(w) V^T in the storage precision.
//
// The rotation of a pair uses the symmetric 2x2 Schur decomposition
// (tan t of the smaller angle; Golub & Van Loan, Matrix Computations,
// Sec. 8.5).  A pair is rotated while |g_pq| > eps sqrt(g_pp g_qq), the
// relative off-diagonal test that gives eigenvalues to high relative accuracy.
#include "common.h"
#include "launch.h"

namespace rpca {
namespace {

constexpr int LD = kEigMaxN + 1;
constexpr double kRotEps = 1.0e-15;
constexpr double kTiny = 1.0e-300;
constexpr int kMaxSweeps = 40;
constexpr int kMaxUpper = (kEigMaxN * (kEigMaxN + 1) / 2 + kEigThreads - 1) / kEigThreads;
constexpr int kMaxFull = (kEigMaxN * kEigMaxN + kEigThreads - 1) / kEigThreads;

__device__ inline bool off_diag_large(double gij, double gii, double gjj) {
  const double a = fabs(gij);
  return a > kTiny && a > kRotEps * sqrt(fabs(gii * gjj));
}

template <typename T>
__global__ void __launch_bounds__(kEigThreads) k_eig(const SolveDesc* __restrict__ descs) {
  __shared__ double G[kEigMaxN * LD];
  __shared__ double V[kEigMaxN * LD];
  __shared__ double C[kEigMaxN * LD];
  __shared__ double al[kEigMaxN], be[kEigMaxN], dg[kEigMaxN], w[kEigMaxN];
  __shared__ int uu[kEigMaxN], vv[kEigMaxN], partner[kEigMaxN];
  __shared__ double scal[kScalars];
  __shared__ int s_go;

  const int tid = threadIdx.x;
  const SolveDesc& d = descs[blockIdx.x];
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

  // Final level of the streaming pass's reduction: group partials added in
  // group order, the Gram straight into LDS.
  {
    const int nblk = gram_blocks((n + 3) >> 2);
    const int nent = kScalars + nblk * 16;
    constexpr int kChunk = 16;
    for (int idx = tid; idx < nent; idx += kEigThreads) {
      double s = 0.0;
      for (int q0 = 0; q0 < d.groups; q0 += kChunk) {
        const int c = min(kChunk, d.groups - q0);
        double v[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q)
          v[q] = q < c ? d.gpartials[static_cast<size_t>(q0 + q) * d.pstride + idx] : 0.0;
#pragma unroll
        for (int q = 0; q < kChunk; ++q)
          if (q < c) s += v[q];
      }
      if (idx < kScalars) {
        scal[idx] = s;
      } else {
        const int g = idx - kScalars;
        const int blk = g >> 4, e = g & 15;
        int bj = 0;
        while ((bj + 1) * (bj + 2) / 2 <= blk) ++bj;
        const int bi = blk - bj * (bj + 1) / 2;
        const int i = 4 * bi + (e >> 2), j = 4 * bj + (e & 3);
        if (i < n && j < n) {
          G[i * LD + j] = s;
          G[j * LD + i] = s;
        }
      }
    }
  }
  __syncthreads();

  if (tid == 0) {
    int go = 0;
    if (kd == 0) {
      st->nX1 = scal[1];
      st->nXF2 = scal[2];
      st->nonfinite = scal[3] > 0.0 ? 1 : 0;
      if (st->nonfinite) {
        st->status = kErrNonfinite;
        st->done = 1;
      } else if (st->nX1 == 0.0) {
        st->status = kOk;
        st->resid = 0.0;
        st->done = 1;
      } else {
        const double mu = d.mu_in > 0.0
                              ? d.mu_in
                              : static_cast<double>(d.m) * static_cast<double>(d.n) / (4.0 * st->nX1);
        const double lam = d.lam_in > 0.0
                               ? d.lam_in
                               : 1.0 / sqrt(static_cast<double>(d.m > d.n ? d.m : d.n));
        st->mu = mu;
        st->imu = 1.0 / mu;
        st->tau = 1.0 / mu;
        st->lam = lam;
        st->gamma = lam / mu;
        go = 1;
      }
    } else {
      st->r2 = scal[0];
      const double rel = sqrt(st->r2) / sqrt(st->nXF2);
      st->resid = rel;
      if (!__builtin_isfinite(st->r2)) {
        st->status = kErrNonfinite;
        st->done = 1;
      } else if (d.tol > 0.0 && rel < d.tol) {
        st->status = kOk;
        st->done = 1;
      } else if (kd >= d.maxit) {
        st->status = kNotConverged;
        st->done = 1;
      } else {
        go = 1;
      }
    }
    s_go = go;
  }
  __syncthreads();
  if (!s_go) return;
  EIG_MARK(0);

  const bool warm = kd > 0;
  const double tau = st->tau;

  // Upper-triangle entries owned by this thread (column-packed order).
  const int nup = n * (n + 1) / 2;
  int ui[kMaxUpper], uj[kMaxUpper];
#pragma unroll
  for (int q = 0; q < kMaxUpper; ++q) {
    const int idx = tid + q * kEigThreads;
    int j = 0;
    if (idx < nup) {
      while ((j + 1) * (j + 2) / 2 <= idx) ++j;
    }
    uj[q] = j;
    ui[q] = idx < nup ? idx - j * (j + 1) / 2 : 0;
  }
  const int nfull = n * n;

  for (int idx = tid; idx < nfull; idx += kEigThreads) {
    const int i = idx / n, j = idx - (idx / n) * n;
    V[i * LD + j] = warm ? d.V[i * nb + j] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  EIG_MARK(1);

  if (warm) {
    // Newton-Schulz: C = V^T V, then V <- V (1.5 I - 0.5 C).
    double cu[kMaxUpper];
#pragma unroll
    for (int q = 0; q < kMaxUpper; ++q) {
      cu[q] = 0.0;
      if (tid + q * kEigThreads < nup) {
        const int i = ui[q], j = uj[q];
        double s = 0.0;
        for (int k = 0; k < n; ++k) s = fma(V[k * LD + i], V[k * LD + j], s);
        cu[q] = s;
      }
    }
#pragma unroll
    for (int q = 0; q < kMaxUpper; ++q) {
      if (tid + q * kEigThreads < nup) {
        C[ui[q] * LD + uj[q]] = cu[q];
        C[uj[q] * LD + ui[q]] = cu[q];
      }
    }
    __syncthreads();
    double vt[kMaxFull];
#pragma unroll
    for (int q = 0; q < kMaxFull; ++q) {
      const int idx = tid + q * kEigThreads;
      vt[q] = 0.0;
      if (idx < nfull) {
        const int i = idx / n, j = idx - (idx / n) * n;
        double s = 1.5 * V[i * LD + j];
        for (int k = 0; k < n; ++k) s = fma(-0.5 * V[i * LD + k], C[k * LD + j], s);
        vt[q] = s;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kMaxFull; ++q) {
      const int idx = tid + q * kEigThreads;
      if (idx < nfull) {
        const int i = idx / n, j = idx - (idx / n) * n;
        V[i * LD + j] = vt[q];
      }
    }
    __syncthreads();

    double tmp[kMaxFull];
#pragma unroll
    for (int q = 0; q < kMaxFull; ++q) {
      const int idx = tid + q * kEigThreads;
      tmp[q] = 0.0;
      if (idx < nfull) {
        const int i = idx / n, j = idx - (idx / n) * n;
        double s = 0.0;
        for (int k = 0; k < n; ++k) s = fma(G[i * LD + k], V[k * LD + j], s);
        tmp[q] = s;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kMaxFull; ++q) {
      const int idx = tid + q * kEigThreads;
      if (idx < nfull) {
        const int i = idx / n, j = idx - (idx / n) * n;
        G[i * LD + j] = tmp[q];  // G now holds W = G V
      }
    }
    __syncthreads();
    double tu[kMaxUpper];
#pragma unroll
    for (int q = 0; q < kMaxUpper; ++q) {
      tu[q] = 0.0;
      if (tid + q * kEigThreads < nup) {
        const int i = ui[q], j = uj[q];
        double s = 0.0;
        for (int k = 0; k < n; ++k) s = fma(V[k * LD + i], G[k * LD + j], s);
        tu[q] = s;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kMaxUpper; ++q) {
      if (tid + q * kEigThreads < nup) {
        G[ui[q] * LD + uj[q]] = tu[q];
        G[uj[q] * LD + ui[q]] = tu[q];
      }
    }
    __syncthreads();
  }
  EIG_MARK(2);

  const int N2 = n + (n & 1);
  int sweeps = 0;
  for (; sweeps < kMaxSweeps && n > 1; ++sweeps) {
    int need = 0;
#pragma unroll
    for (int q = 0; q < kMaxUpper; ++q) {
      if (tid + q * kEigThreads < nup && ui[q] < uj[q]) {
        const int i = ui[q], j = uj[q];
        if (off_diag_large(G[i * LD + j], G[i * LD + i], G[j * LD + j])) need = 1;
      }
    }
    if (!__syncthreads_or(need)) break;
    for (int r = 0; r < N2 - 1; ++r) {
      if (tid < N2 / 2) {
        int a, b;
        if (tid == 0) {
          a = N2 - 1;
          b = r;
        } else {
          a = (r + tid) % (N2 - 1);
          b = (r - tid + N2 - 1) % (N2 - 1);
        }
        const int p = a < b ? a : b;
        const int q = a < b ? b : a;
        bool rot = false;
        if (q < n) {
          const double gpp = G[p * LD + p], gqq = G[q * LD + q], gpq = G[p * LD + q];
          if (off_diag_large(gpq, gpp, gqq)) {
            const double th = (gqq - gpp) / (2.0 * gpq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
            const double c = 1.0 / sqrt(1.0 + t * t);
            const double s = t * c;
            uu[p] = p; vv[p] = q; al[p] = c; be[p] = -s; dg[p] = -t * gpq; partner[p] = q;
            uu[q] = p; vv[q] = q; al[q] = s; be[q] = c;  dg[q] = t * gpq;  partner[q] = p;
            rot = true;
          }
        }
        if (!rot) {
          if (p < n) { uu[p] = p; vv[p] = p; al[p] = 1.0; be[p] = 0.0; dg[p] = 0.0; partner[p] = -1; }
          if (q < n) { uu[q] = q; vv[q] = q; al[q] = 1.0; be[q] = 0.0; dg[q] = 0.0; partner[q] = -1; }
        }
      }
      __syncthreads();
      double gn[kMaxUpper], vn[kMaxFull];
#pragma unroll
      for (int q = 0; q < kMaxUpper; ++q) {
        gn[q] = 0.0;
        if (tid + q * kEigThreads < nup) {
          const int i = ui[q], j = uj[q];
          if (i == j) {
            gn[q] = G[i * LD + i] + dg[i];
          } else if (partner[i] == j) {
            gn[q] = 0.0;
          } else {
            const int ua = uu[i], va = vv[i], ub = uu[j], vb = vv[j];
            const double ai = al[i], bi = be[i], aj = al[j], bj = be[j];
            double s = ai * aj * G[ua * LD + ub];
            s = fma(ai * bj, G[ua * LD + vb], s);
            s = fma(bi * aj, G[va * LD + ub], s);
            s = fma(bi * bj, G[va * LD + vb], s);
            gn[q] = s;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < kMaxFull; ++q) {
        vn[q] = 0.0;
        const int idx = tid + q * kEigThreads;
        if (idx < nfull) {
          const int rr = idx / n, j = idx - (idx / n) * n;
          vn[q] = fma(al[j], V[rr * LD + uu[j]], be[j] * V[rr * LD + vv[j]]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kMaxUpper; ++q) {
        if (tid + q * kEigThreads < nup) {
          G[ui[q] * LD + uj[q]] = gn[q];
          G[uj[q] * LD + ui[q]] = gn[q];
        }
      }
#pragma unroll
      for (int q = 0; q < kMaxFull; ++q) {
        const int idx = tid + q * kEigThreads;
        if (idx < nfull) {
          const int rr = idx / n, j = idx - (idx / n) * n;
          V[rr * LD + j] = vn[q];
        }
      }
      __syncthreads();
    }
  }

  EIG_MARK(3);
  // SVT weights from the eigenvalues sigma_i^2 of A^T A.
  if (tid < n) {
    const double sg = sqrt(fmax(G[tid * LD + tid], 0.0));
    w[tid] = sg > tau ? (sg - tau) / sg : 0.0;
  }
  __syncthreads();

  T* __restrict__ Pd = static_cast<T*>(d.P);
  for (int idx = tid; idx < nb * nb; idx += kEigThreads) {
    const int i = idx / nb, j = idx - (idx / nb) * nb;
    double s = 0.0;
    if (i < n && j < n) {
      for (int k = 0; k < n; ++k) {
        const double wk = w[k];
        if (wk != 0.0) s = fma(V[i * LD + k] * wk, V[j * LD + k], s);
      }
    }
    Pd[idx] = static_cast<T>(s);
  }
  for (int idx = tid; idx < nfull; idx += kEigThreads) {
    const int i = idx / n, j = idx - (idx / n) * n;
    d.V[i * nb + j] = V[i * LD + j];
  }
  EIG_MARK(4);
  if (tid == 0) {
    int rank = 0;
    for (int k = 0; k < n; ++k) rank += w[k] != 0.0 ? 1 : 0;
    st->rank = rank;
    st->sweeps = sweeps;
    st->sweeps_total += sweeps;
    st->iter = st->iter + 1;
  }
}

}  // namespace

hipError_t launch_eig(int dtype, int grid, hipStream_t stream, const SolveDesc* descs) {
  if (grid <= 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(k_eig<double>, dim3(grid), dim3(kEigThreads), 0, stream, descs);
  else
    hipLaunchKernelGGL(k_eig<float>, dim3(grid), dim3(kEigThreads), 0, stream, descs);
  return hipGetLastError();
}

}  // namespace rpca
