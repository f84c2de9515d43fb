// Workgroup-cooperative small dense linear algebra in FP64 for gfx950.
//
// Every routine is executed by all threads of one workgroup (blockDim.x a
// multiple of 64), works on strided views that may point to LDS or global
// memory, and ends with a workgroup barrier so that its results are visible
// to every thread.  Sizes are runtime values; the callers keep them within
// the LDS capacities of the task interpreter.
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"

namespace h2 {

struct MV {
  double *p;
  int rs, cs;
  // offsets inside one slot/buffer view stay below 2^31 (32-bit arithmetic)
  __device__ __forceinline__ double &operator()(int i, int j) const { return p[i * rs + j * cs]; }
};
__device__ __forceinline__ MV mv_col(double *p, int ld) { return MV{p, 1, ld}; }
__device__ __forceinline__ MV mv_row(double *p, int ld) { return MV{p, ld, 1}; }
__device__ __forceinline__ MV mv_t(MV a) { return MV{a.p, a.cs, a.rs}; }
__device__ __forceinline__ MV mv_at(MV a, int i, int j) { return MV{a.p + i * a.rs + j * a.cs, a.rs, a.cs}; }

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }
__device__ __forceinline__ int num_waves() { return blockDim.x >> 6; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Register-to-register data movement between lanes (DPP) for doubles.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over aligned groups of g lanes (g in {1, 2, 4, 8, 16}); every lane of
// the group receives the sum.  Butterfly: xor 1, xor 2 (quad_perm), then
// half-row and row mirrors.
__device__ __forceinline__ double group_sum(double v, int g) {
  if (g >= 2) v += dpp_d<0xB1>(v);     // quad_perm [1,0,3,2]
  if (g >= 4) v += dpp_d<0x4E>(v);     // quad_perm [2,3,0,1]
  if (g >= 8) v += dpp_d<0x141>(v);    // row_half_mirror
  if (g >= 16) v += dpp_d<0x140>(v);   // row_mirror
  return v;
}

// Sum of one value per thread over the workgroup; red holds >= 16 doubles.
__device__ __forceinline__ double wg_sum(double v, double *red) {
  v = wave_sum(v);
  __syncthreads();
  if (lane_id() == 0) red[wave_id()] = v;
  __syncthreads();
  double s = 0;
  for (int w = 0; w < num_waves(); ++w) s += red[w];
  __syncthreads();
  return s;
}

__device__ __forceinline__ int wg_or(int v, int *ired) {
  __syncthreads();
  if (threadIdx.x == 0) *ired = 0;
  __syncthreads();
  if (v) *ired = 1;
  __syncthreads();
  int r = *ired;
  __syncthreads();
  return r;
}

// C (m x n) = alpha * A (m x k) * B (k x n) + beta * C.  C must not alias A/B.
// Thread t computes the entries t, t + NT, ... in column-major order; the
// row/column of the next entry is advanced without integer division.
__device__ void wg_gemm(int m, int n, int k, double alpha, MV A, MV B, double beta, MV C) {
  if (m > 0 && n > 0) {
    const int nt = blockDim.x;
    int i = threadIdx.x % m, j = threadIdx.x / m;
    const int di = nt % m, dj = nt / m;
    while (j < n) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) s = fma(A(i, l), B(l, j), s);
      C(i, j) = (beta == 0.0 ? 0.0 : beta * C(i, j)) + alpha * s;
      i += di; j += dj;
      if (i >= m) { i -= m; ++j; }
    }
  }
  __syncthreads();
}

// Division-free walk over the entries of an m x n matrix: a thread starts at
// entry `start` (column-major) and advances by `step` entries.
struct Walk2 {
  int i, j, di, dj, m;
  __device__ __forceinline__ Walk2(int start, int step, int m_) : m(m_) {
    i = start % m; j = start / m; di = step % m; dj = step / m;
  }
  __device__ __forceinline__ void next() { i += di; j += dj; if (i >= m) { i -= m; ++j; } }
};

__device__ void wg_copy(int m, int n, MV src, MV dst) {
  if (m > 0 && n > 0)
    for (Walk2 w(threadIdx.x, blockDim.x, m); w.j < n; w.next()) dst(w.i, w.j) = src(w.i, w.j);
  __syncthreads();
}

__device__ void wg_fill(int m, int n, MV dst, double v) {
  if (m > 0 && n > 0)
    for (Walk2 w(threadIdx.x, blockDim.x, m); w.j < n; w.next()) dst(w.i, w.j) = v;
  __syncthreads();
}

// Householder QR of A (m x n) in place (LAPACK dlarfg convention).  On exit
// the upper triangle of the first min(m,n) rows holds R, the strictly lower
// part holds the Householder vectors (unit first entry implied) and tau[j]
// (if tau != nullptr) the scalar factors.  red: >= 4 doubles of scratch.
__device__ void wg_qr(int m, int n, MV A, double *tau, double *red) {
  const int kmax = m < n ? m : n;
  const int lane = lane_id(), wave = wave_id(), nw = num_waves();
  for (int j = 0; j < kmax; ++j) {
    if (wave == 0) {
      double s = 0.0;
      for (int i = j + 1 + lane; i < m; i += 64) {
        const double v = A(i, j);
        s = fma(v, v, s);
      }
      s = wave_sum(s);
      if (lane == 0) {
        const double alpha = A(j, j);
        double t = 0.0, beta = alpha, scale = 0.0;
        if (s > 0.0) {
          const double nrm = sqrt(fma(alpha, alpha, s));
          beta = alpha >= 0.0 ? -nrm : nrm;
          t = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
        red[0] = t; red[1] = beta; red[2] = scale;
      }
    }
    __syncthreads();
    const double t = red[0], beta = red[1], scale = red[2];
    if (t != 0.0) {
      for (int i = j + 1 + threadIdx.x; i < m; i += blockDim.x) A(i, j) *= scale;
      __syncthreads();
      for (int c = j + 1 + wave; c < n; c += nw) {
        double w = 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) w = fma(A(i, j), A(i, c), w);
        w = wave_sum(w);
        w = t * (w + A(j, c));
        for (int i = j + 1 + lane; i < m; i += 64) A(i, c) = fma(-w, A(i, j), A(i, c));
        if (lane == 0) A(j, c) -= w;
      }
      if (threadIdx.x == 0) A(j, j) = beta;
    } else {
      for (int i = j + 1 + threadIdx.x; i < m; i += blockDim.x) A(i, j) = 0.0;
    }
    if (tau != nullptr && threadIdx.x == 0) tau[j] = t;
    __syncthreads();
  }
}

// Copy R (rows min(m,n), upper triangular/trapezoidal) of a factorised A to R.
__device__ void wg_extract_r(int m, int n, MV A, MV R) {
  const int kmax = m < n ? m : n;
  const int tot = kmax * n;
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int i = idx % kmax, j = idx / kmax;
    R(i, j) = (j >= i) ? A(i, j) : 0.0;
  }
  __syncthreads();
}

// Zero the strictly lower part of the first min(m,n) rows (turn a factorised
// A into [R; junk] with R clean).
__device__ void wg_clean_r(int m, int n, MV A) {
  const int kmax = m < n ? m : n;
  const int tot = kmax * kmax;
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int i = idx % kmax, j = idx / kmax;
    if (i > j) A(i, j) = 0.0;
  }
  __syncthreads();
}

// Explicit Q (m x q, q = min(m,n)) of a factorised A: Q = H_0 ... H_{q-1} [I; 0].
__device__ void wg_form_q(int m, int n, MV A, const double *tau, MV Q) {
  const int q = m < n ? m : n;
  const int lane = lane_id(), wave = wave_id(), nw = num_waves();
  const int tot = m * q;
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int i = idx % m, j = idx / m;
    Q(i, j) = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = q - 1; j >= 0; --j) {
    const double t = tau[j];
    if (t != 0.0) {
      for (int c = j + wave; c < q; c += nw) {
        double w = 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) w = fma(A(i, j), Q(i, c), w);
        w = wave_sum(w);
        w = t * (w + Q(j, c));
        for (int i = j + 1 + lane; i < m; i += 64) Q(i, c) = fma(-w, A(i, j), Q(i, c));
        if (lane == 0) Q(j, c) -= w;
      }
    }
    __syncthreads();
  }
}

// Rotation that makes columns a, b orthogonal given alpha = |a|^2,
// beta = |b|^2, gamma = a.b: with d = beta - alpha,
// t = 2 gamma sgn(d) / (|d| + sqrt(d^2 + 4 gamma^2)) (the smaller root of
// t^2 + 2 zeta t - 1 = 0, zeta = d / (2 gamma)), c = 1/sqrt(1+t^2), s = c t.
__device__ __forceinline__ void jacobi_rotation(double al, double be, double ga, double &c, double &s) {
  const double d = be - al;
  const double t = (d >= 0.0 ? 2.0 * ga : -2.0 * ga) / (fabs(d) + sqrt(fma(d, d, 4.0 * ga * ga)));
  c = __builtin_amdgcn_rsq(1.0 + t * t);
  c = c * fma(-0.5 * (1.0 + t * t) * c, c, 1.5);   // one Newton step on the hardware rsqrt
  s = c * t;
}

// One-sided (Hestenes) Jacobi: rotate the columns of G (m x n) until they are
// mutually orthogonal; the same rotations are applied to J (n x n, if not
// null), which then holds the right singular vectors (G_in J = G_out).
// Pairs are visited in round-robin order; all n/2 disjoint pairs of a round
// are processed at once, each by a group of g lanes (g a power of two, the
// groups aligned inside a wave), with one workgroup barrier per round.
__device__ int wg_jacobi(int m, int n, MV G, MV *J, int *sflag) {
  if (n < 2) { __syncthreads(); return 0; }
  int sweeps = 0;
  const int np = n + (n & 1);
  const int npairs = np / 2;
  int g = 64;
  while (g > 1 && npairs * g > (int)blockDim.x) g >>= 1;
  const int gid = threadIdx.x / g, gl = threadIdx.x % g, ngroups = blockDim.x / g;
  const double tol = 4.0e-16 * (double)(m > 8 ? m : 8), tol2 = tol * tol;
  for (int sweep = 0; sweep < 60; ++sweep) {
    __syncthreads();
    if (threadIdx.x == 0) *sflag = 0;
    __syncthreads();
    for (int r = 0; r < np - 1; ++r) {
      for (int p = gid; p < npairs; p += ngroups) {
        int a, b;
        if (p == 0) { a = np - 1; b = r; }
        else { a = (r + p) % (np - 1); b = (r - p + np - 1) % (np - 1); }
        if (a > b) { const int tt = a; a = b; b = tt; }
        if (b >= n) continue;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = gl; i < m; i += g) {
          const double x = G(i, a), y = G(i, b);
          al = fma(x, x, al); be = fma(y, y, be); ga = fma(x, y, ga);
        }
        for (int o = g >> 1; o > 0; o >>= 1) {
          al += __shfl_xor(al, o, 64);
          be += __shfl_xor(be, o, 64);
          ga += __shfl_xor(ga, o, 64);
        }
        if (ga != 0.0 && ga * ga > tol2 * (al * be)) {
          double c, s;
          jacobi_rotation(al, be, ga, c, s);
          for (int i = gl; i < m; i += g) {
            const double x = G(i, a), y = G(i, b);
            G(i, a) = c * x - s * y;
            G(i, b) = s * x + c * y;
          }
          if (J != nullptr) {
            MV Jm = *J;
            for (int i = gl; i < n; i += g) {
              const double x = Jm(i, a), y = Jm(i, b);
              Jm(i, a) = c * x - s * y;
              Jm(i, b) = s * x + c * y;
            }
          }
          if (gl == 0) *sflag = 1;
        }
      }
      __syncthreads();
    }
    ++sweeps;
    if (*sflag == 0) break;
  }
  __syncthreads();
  return sweeps;
}

// Single-wave one-sided Jacobi (same rotations and ordering as wg_jacobi):
// executed by the 64 lanes of one wave, no workgroup barrier.  Each of the
// n/2 pairs of a round is handled by a group of g lanes (g = largest power
// of two with pairs * g <= 64); the wave's LDS accesses complete in program
// order, so rounds only need a compiler scheduling barrier.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ int wave_jacobi(int m, int n, MV G, MV *J) {
  if (n < 2) return 0;
  const int lane = lane_id();
  const int np = n + (n & 1);
  const int npairs = np / 2;
  int g = 16;
  while (g > 1 && npairs * g > 64) g >>= 1;
  const int gid = lane / g, gl = lane % g, ngroups = 64 / g;
  const double tol = 4.0e-16 * (double)(m > 8 ? m : 8), tol2 = tol * tol;
  int sweeps = 0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    int rotated = 0;
    for (int r = 0; r < np - 1; ++r) {
      for (int p = gid; p < npairs; p += ngroups) {
        int a, b;
        if (p == 0) { a = np - 1; b = r; }
        else {
          a = r + p; if (a >= np - 1) a -= np - 1;
          b = r - p + np - 1; if (b >= np - 1) b -= np - 1;
        }
        if (a > b) { const int tt = a; a = b; b = tt; }
        double al = 0.0, be = 0.0, ga = 0.0;
        if (b < n) {
          for (int i = gl; i < m; i += g) {
            const double x = G(i, a), y = G(i, b);
            al = fma(x, x, al); be = fma(y, y, be); ga = fma(x, y, ga);
          }
        }
        // all lanes take part in the DPP reduction (dummy pairs add zeros)
        al = group_sum(al, g); be = group_sum(be, g); ga = group_sum(ga, g);
        if (b < n && ga != 0.0 && ga * ga > tol2 * (al * be)) {
          double c, s;
          jacobi_rotation(al, be, ga, c, s);
          for (int i = gl; i < m; i += g) {
            const double x = G(i, a), y = G(i, b);
            G(i, a) = c * x - s * y;
            G(i, b) = s * x + c * y;
          }
          if (J != nullptr) {
            MV Jm = *J;
            for (int i = gl; i < n; i += g) {
              const double x = Jm(i, a), y = Jm(i, b);
              Jm(i, a) = c * x - s * y;
              Jm(i, b) = s * x + c * y;
            }
          }
          rotated = 1;
        }
      }
      wave_sync();
    }
    ++sweeps;
    if (__ballot(rotated) == 0) break;
  }
  return sweeps;
}

// ---------------------------------------------------------------------------
// Wave-level versions: executed by the 64 lanes of one wave, no workgroup
// barrier, so several waves can work on independent clusters at once.

__device__ __forceinline__ double wave_sum64(double v) {
  v = group_sum(v, 16);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// C (m x n) = alpha * A (m x k) * B (k x n) + beta * C (no aliasing).
__device__ void wv_gemm(int m, int n, int k, double alpha, MV A, MV B, double beta, MV C) {
  if (m > 0 && n > 0) {
    const int lane = lane_id();
    int i = lane % m, j = lane / m;
    const int di = 64 % m, dj = 64 / m;
    while (j < n) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) s = fma(A(i, l), B(l, j), s);
      C(i, j) = (beta == 0.0 ? 0.0 : beta * C(i, j)) + alpha * s;
      i += di; j += dj;
      if (i >= m) { i -= m; ++j; }
    }
  }
  wave_sync();
}

// Householder QR in place (as wg_qr): the column norm is a wave reduction,
// the update of the trailing columns runs one lane per column.
__device__ void wv_qr(int m, int n, MV A, double *tau) {
  const int lane = lane_id();
  const int kmax = m < n ? m : n;
  for (int j = 0; j < kmax; ++j) {
    double s = 0.0;
    for (int i = j + 1 + lane; i < m; i += 64) { const double v = A(i, j); s = fma(v, v, s); }
    s = wave_sum64(s);
    const double alpha = A(j, j);
    double t = 0.0, beta = alpha, scale = 0.0;
    if (s > 0.0) {
      const double nrm = sqrt(fma(alpha, alpha, s));
      beta = alpha >= 0.0 ? -nrm : nrm;
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    wave_sync();
    if (t != 0.0) {
      for (int i = j + 1 + lane; i < m; i += 64) A(i, j) *= scale;
      wave_sync();
      for (int c = j + 1 + lane; c < n; c += 64) {
        double w = A(j, c);
        for (int i = j + 1; i < m; ++i) w = fma(A(i, j), A(i, c), w);
        w *= t;
        A(j, c) -= w;
        for (int i = j + 1; i < m; ++i) A(i, c) = fma(-w, A(i, j), A(i, c));
      }
      wave_sync();
      if (lane == 0) A(j, j) = beta;
    } else {
      for (int i = j + 1 + lane; i < m; i += 64) A(i, j) = 0.0;
    }
    if (tau != nullptr && lane == 0) tau[j] = t;
    wave_sync();
  }
}

// Column norms (one lane per column) and descending ranking, wave level.
__device__ void wv_colnorms_sorted(int m, int n, MV G, double *sig, int *ord) {
  const int lane = lane_id();
  for (int c = lane; c < n; c += 64) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) { const double x = G(i, c); s = fma(x, x, s); }
    sig[c] = sqrt(s);
  }
  wave_sync();
  for (int c = lane; c < n; c += 64) {
    const double v = sig[c];
    int rank = 0;
    for (int c2 = 0; c2 < n; ++c2) {
      const double w = sig[c2];
      rank += (w > v || (w == v && c2 < c)) ? 1 : 0;
    }
    ord[rank] = c;
  }
  wave_sync();
}

// Column norms of G (m x n) into sig[0..n) and the permutation ord[0..n)
// sorting them in descending order (ties by index).  One thread per column
// for the norms, then every column computes its own rank.
__device__ void wg_colnorms_sorted(int m, int n, MV G, double *sig, int *ord) {
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) { const double x = G(i, c); s = fma(x, x, s); }
    sig[c] = sqrt(s);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const double v = sig[c];
    int rank = 0;
    for (int c2 = 0; c2 < n; ++c2) {
      const double w = sig[c2];
      rank += (w > v || (w == v && c2 < c)) ? 1 : 0;
    }
    ord[rank] = c;
  }
  __syncthreads();
}

// Lower Cholesky factor of A (n x n) in place using the lower triangle;
// the strict upper triangle is zeroed.  Returns 0 or (j+1) for a
// non-positive pivot j.
__device__ int wg_potrf(int n, MV A, int *iflag) {
  if (threadIdx.x == 0) *iflag = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      const double d = A(j, j);
      if (!(d > 0.0)) { if (*iflag == 0) *iflag = j + 1; A(j, j) = 1.0; }
      else A(j, j) = sqrt(d);
    }
    __syncthreads();
    const double djj = A(j, j);
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) A(i, j) /= djj;
    __syncthreads();
    const int rem = n - j - 1;
    for (int idx = threadIdx.x; idx < rem * rem; idx += blockDim.x) {
      const int i = j + 1 + idx % rem, c = j + 1 + idx / rem;
      if (c <= i) A(i, c) = fma(-A(i, j), A(c, j), A(i, c));
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx % n, c = idx / n;
    if (c > i) A(i, c) = 0.0;
  }
  __syncthreads();
  const int r = *iflag;
  __syncthreads();
  return r;
}

// One wave solves L x = b (trans = 0) or L^T x = b (trans = 1) for lower
// triangular L (n <= 64): lane i keeps row i (or column i) of L in
// registers and the solution is propagated with shuffles.
template <int NMAX>
__device__ __forceinline__ void wave_load_tri(int n, MV L, int trans, double (&row)[NMAX]) {
  const int lane = lane_id();
#pragma unroll
  for (int l = 0; l < NMAX; ++l) {
    double v = 0.0;
    if (lane < n && l < n) v = trans ? L(l, lane) : L(lane, l);
    row[l] = v;
  }
}

template <int NMAX>
__device__ __forceinline__ double wave_tri_solve(int n, const double (&row)[NMAX], int trans, double b) {
  const int lane = lane_id();
  // fully unrolled with static indices into row[] (no dynamic register
  // indexing); steps j >= n are skipped by a uniform predicate
  if (!trans) {
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
      if (j < n) {
        const double xj = __shfl(b, j, 64) / __shfl(row[j], j, 64);
        if (lane == j) b = xj;
        else if (lane > j) b = fma(-row[j], xj, b);
      }
    }
  } else {
#pragma unroll
    for (int j = NMAX - 1; j >= 0; --j) {
      if (j < n) {
        const double xj = __shfl(b, j, 64) / __shfl(row[j], j, 64);
        if (lane == j) b = xj;
        else if (lane < j) b = fma(-row[j], xj, b);
      }
    }
  }
  return b;
}

// X (m x n) <- X L^{-T} for lower triangular L (n x n, n <= LS): every row x
// of X solves L x^T = row^T; one wave per row.
__device__ void wg_trsm_right_lt(int m, int n, MV L, MV X) {
  double row[LS];
  wave_load_tri<LS>(n, L, 0, row);
  const int lane = lane_id();
  for (int i = wave_id(); i < m; i += num_waves()) {
    double b = lane < n ? X(i, lane) : 0.0;
    b = wave_tri_solve<LS>(n, row, 0, b);
    if (lane < n) X(i, lane) = b;
  }
  __syncthreads();
}

// B (n x m) <- L^{-1} B (trans = 0) or L^{-T} B (trans = 1), n <= LS; one
// wave per column of B.
__device__ void wg_trsv_lower(int n, int m, MV L, MV B, int trans) {
  double row[LS];
  wave_load_tri<LS>(n, L, trans, row);
  const int lane = lane_id();
  for (int c = wave_id(); c < m; c += num_waves()) {
    double b = lane < n ? B(lane, c) : 0.0;
    b = wave_tri_solve<LS>(n, row, trans, b);
    if (lane < n) B(lane, c) = b;
  }
  __syncthreads();
}

}  // namespace h2
