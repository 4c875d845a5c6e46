// Pieces shared by the eigensolve kernels (paper Sec. II-A, Eq. 4): the
// Jacobi rotation of a pair, the round-robin pairing, fixed-order dot
// products and the per-iteration control step.
#pragma once

#include "common.h"

namespace rpca {
namespace eigk {

constexpr double kTiny2 = 1.0e-300;
constexpr int kMaxSweeps = 40;

template <typename T>
struct RotEps;
template <>
struct RotEps<double> {
  static constexpr double eps2 = 1.0e-30;
};
template <>
struct RotEps<float> {
  static constexpr double eps2 = 1.0e-16;
};

template <typename T>
__device__ inline bool off_diag_large(double gij, double gii, double gjj) {
  const double a2 = gij * gij;
  return a2 > kTiny2 && a2 > RotEps<T>::eps2 * fabs(gii * gjj);
}

// Round-robin pairing of round r (0 <= r < N2-1) over N2 (even) indices:
// pair 0 is (N2-1, r), pair k >= 1 is ((r+k) mod M, (r-k) mod M), M = N2-1.
__device__ inline void pair_indices(int r, int k, int N2, int& p, int& q) {
  const int M = N2 - 1;
  int a, b;
  if (k == 0) {
    a = N2 - 1;
    b = r;
  } else {
    a = r + k;
    if (a >= M) a -= M;
    b = r - k;
    if (b < 0) b += M;
  }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// Per-round column table of J, written by the threads that compute the
// round's rotations: for index i, column i of J is a_i e_u + b_i e_v with
// (u, v) the pair containing i, packed as u | v << 8 | rotated << 16, (a_i,
// b_i) stored together (one 16-byte read), and dg_i the exact shift of the
// diagonal entry g_ii (-t g_pq for p, +t g_pq for q).  An index paired with
// the padding index gets the identity column.
__device__ inline void set_pair_columns(int p, int q, int n, double c, double s, double dt,
                                        int* cu, double2* cab, double* cd) {
  if (q >= n) {
    cu[p] = p | (p << 8);
    cab[p] = make_double2(1.0, 0.0);
    cd[p] = 0.0;
    return;
  }
  const int packed = p | (q << 8) | (s != 0.0 ? (1 << 16) : 0);
  cu[p] = packed;
  cab[p] = make_double2(c, -s);
  cd[p] = -dt;
  cu[q] = packed;
  cab[q] = make_double2(s, c);
  cd[q] = dt;
}

// Entry (i, j) of J^T G J from the column table (G with leading dimension LD).
template <int LD>
__device__ inline double rotated_entry(int i, int j, const double* G, const int* cu,
                                       const double2* cab, const double* cd) {
  const int pi = cu[i], pj = cu[j];
  const int ui = pi & 0xff, vi = (pi >> 8) & 0xff;
  const int uj = pj & 0xff, vj = (pj >> 8) & 0xff;
  const double2 abi = cab[i], abj = cab[j];
  const double ai = abi.x, bi = abi.y, aj = abj.x, bj = abj.y;
  double gen = ai * aj * G[ui * LD + uj];
  gen = fma(ai * bj, G[ui * LD + vj], gen);
  gen = fma(bi * aj, G[vi * LD + uj], gen);
  gen = fma(bi * bj, G[vi * LD + vj], gen);
  const double diag = G[i * LD + i] + cd[i];
  const bool same_rotated_pair = (pi >> 16) != 0 && (pi & 0xffff) == (pj & 0xffff);
  return i == j ? diag : (same_rotated_pair ? 0.0 : gen);
}

// 1/x and 1/sqrt(x) for positive normal x: the hardware estimate refined by
// two Newton steps (each doubles the number of correct bits).
__device__ inline double rcp_pos(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * fma(-x, r, 2.0);
  r = r * fma(-x, r, 2.0);
  return r;
}
__device__ inline double rsqrt_pos(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}

// Rotation of one pair from the entries of G.
template <typename T>
__device__ inline void make_rotation(double gpp, double gqq, double gpq, double& c, double& s,
                                     double& dt) {
  if (off_diag_large<T>(gpq, gpp, gqq)) {
    const double d = gqq - gpp;
    const double h2 = fma(d, d, 4.0 * gpq * gpq);   // > 0 since gpq != 0
    const double h = h2 * rsqrt_pos(h2);
    double t = 2.0 * gpq * rcp_pos(fabs(d) + h);
    if (d < 0.0) t = -t;
    c = rsqrt_pos(fma(t, t, 1.0));
    s = t * c;
    dt = t * gpq;
  } else {
    c = 1.0;
    s = 0.0;
    dt = 0.0;
  }
}

// Dot product over the zero-padded length NMAX with four independent
// partial sums (fixed trip count, so every load can be in flight at once).
template <int NMAX, typename F>
__device__ inline double dot4(F&& term) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll 4
  for (int k = 0; k < NMAX; k += 4) {
    s0 = term(k + 0, s0);
    s1 = term(k + 1, s1);
    s2 = term(k + 2, s2);
    s3 = term(k + 3, s3);
  }
  return (s0 + s1) + (s2 + s3);
}

// The same sum over the first len terms only (len a multiple of 4, at most
// NMAX): used where the terms past the matrix size n are exact zeros, so the
// value is the same and the padding costs nothing.
template <int NMAX, typename F>
__device__ inline double dot4n(int len, F&& term) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll 2
  for (int k = 0; k < len; k += 4) {
    s0 = term(k + 0, s0);
    s1 = term(k + 1, s1);
    s2 = term(k + 2, s2);
    s3 = term(k + 3, s3);
  }
  return (s0 + s1) + (s2 + s3);
}

// Control step of an eigensolve launch, run by one thread after the
// reduction has put the pass's scalars in scal (r2, sum|X|, sum X^2,
// non-finite count).  At the first step it records the norms of X and fixes
// mu and lambda (Sec. II-A); afterwards it applies the stopping test of the
// pass that just ran, ||X - L - S||_F < tol ||X||_F, and the iteration cap.
// A solve with a given start (S0, Y0) stops after fixing mu (the Gram of its
// first iterate needs mu) and eigensolves at its next launch.
// nXF2_prev and tau_prev are the state's ||X||_F^2 and tau as the previous
// launch left them (read early by the caller); tau_out receives this launch's
// threshold tau = 1/mu.
// Returns 1 when the eigensolve of this launch goes ahead.
__device__ inline int control_step(const SolveDesc& d, SolveState* st, const double* scal, int kd,
                                   double nXF2_prev, double tau_prev, double& tau_out) {
  int go = 0;
  tau_out = tau_prev;
  if (kd == 0 && d.warm && st->warm_stage == 1) {
    // given start: the reduced Gram is that of A_1 = X - S0 + Y0/mu (the
    // norms and mu were fixed by the previous launch)
    st->warm_stage = 2;
    go = 1;
  } else if (kd == 0) {
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
      tau_out = 1.0 / mu;
      st->lam = lam;
      st->gamma = lam / mu;
      // a given start needs one more pass for the Gram of A_1 before the
      // first eigensolve
      st->warm_stage = d.warm ? 1 : 0;
      go = d.warm ? 0 : 1;
    }
  } else {
    st->r2 = scal[0];
    const double rel = sqrt(scal[0]) / sqrt(nXF2_prev);
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
  return go;
}

}  // namespace eigk
}  // namespace rpca
