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

// Value of lane 0 in every lane (two v_readlane).
__device__ __forceinline__ double bcast_lane0(double v) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 0);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 0);
  return __hiloint2double(hi, lo);
}

// 1/x and sqrt(x) (x > 0, normal range) from the hardware approximations,
// each refined by two Newton steps (relative error a few ulp).
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * fma(-x, y, 2.0);
  y = y * fma(-x, y, 2.0);
  return y;
}
__device__ __forceinline__ double sqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  y = y * fma(-0.5 * x * y, y, 1.5);
  const double r = x * y;
  return fma(0.5 * y, fma(-r, r, x), r);   // one correction of the root itself
}

// acc + sum_{l = lo}^{hi-1} a(l) b(l), accumulated in ascending order.  The
// loads are issued in chunks of U (indices past the end clamped to hi-1 and
// their products dropped), so that a chunk costs one memory latency; a plain
// loop with a run-time trip count waits for every load.
template <int U = 4, class FA, class FB>
__device__ __forceinline__ double dotc(int lo, int hi, FA a, FB b, double acc) {
  for (int l0 = lo; l0 < hi; l0 += U) {
    double x[U], y[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int l = l0 + u < hi ? l0 + u : hi - 1;
      x[u] = a(l);
      y[u] = b(l);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc = fma(l0 + u < hi ? x[u] : 0.0, y[u], acc);
  }
  return acc;
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

// Compile-time group size version for three values at once (the levels of
// the three butterflies are interleaved, no branches).
template <int G>
__device__ __forceinline__ void group_sum3(double &a, double &b, double &c) {
  if (G >= 2) { const double x = dpp_d<0xB1>(a), y = dpp_d<0xB1>(b), z = dpp_d<0xB1>(c); a += x; b += y; c += z; }
  if (G >= 4) { const double x = dpp_d<0x4E>(a), y = dpp_d<0x4E>(b), z = dpp_d<0x4E>(c); a += x; b += y; c += z; }
  if (G >= 8) { const double x = dpp_d<0x141>(a), y = dpp_d<0x141>(b), z = dpp_d<0x141>(c); a += x; b += y; c += z; }
  if (G >= 16) { const double x = dpp_d<0x140>(a), y = dpp_d<0x140>(b), z = dpp_d<0x140>(c); a += x; b += y; c += z; }
}
template <int G>
__device__ __forceinline__ double group_sum_t(double a) {
  if (G >= 2) a += dpp_d<0xB1>(a);
  if (G >= 4) a += dpp_d<0x4E>(a);
  if (G >= 8) a += dpp_d<0x141>(a);
  if (G >= 16) a += dpp_d<0x140>(a);
  return a;
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
// entry `start` (column-major) and advances by `step` entries.  Needs m > 0
// (callers skip empty row ranges).
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

// Rotation for the wave-level sweeps: t from the hardware reciprocal and
// reciprocal square root, each refined by one Newton step; c = 1/sqrt(1+t^2)
// refined the same way so that c^2 + s^2 = 1 to working precision (the
// accuracy of t only affects the convergence speed).
__device__ __forceinline__ void jacobi_rotation_fast(double al, double be, double ga, double &c,
                                                     double &s) {
  const double d = be - al;
  const double h = fma(d, d, 4.0 * ga * ga);
  double y = __builtin_amdgcn_rsq(h);
  y = y * fma(-0.5 * h * y, y, 1.5);
  const double den = fabs(d) + h * y;               // |d| + sqrt(h)
  double z = __builtin_amdgcn_rcp(den);
  z = z * fma(-den, z, 2.0);
  const double t = (d >= 0.0 ? 2.0 * ga : -2.0 * ga) * z;
  const double u = fma(t, t, 1.0);
  c = __builtin_amdgcn_rsq(u);
  c = c * fma(-0.5 * u * c, c, 1.5);
  s = c * t;
}

// One-sided Jacobi on G (m x n), one wave, J (n x n) accumulating the
// rotations when non-null.  Round-robin pairing; each lane group of g lanes
// owns one pair of a round and keeps its RPL rows of both columns in
// registers between the dot products and the rotation.  Row indices past the
// end are clamped to the last row: such lanes load that row, contribute zero
// to the dot products and store the same values as the lane that owns it, so
// the loads and stores need no branches (a branch per row makes the compiler
// wait for every LDS store).  Stops after a sweep without rotation, or after
// a sweep whose largest rotated relative off-diagonal gamma^2/(alpha beta)
// stayed below 1e-14: with quadratic convergence the next sweep would rotate
// by angles of order 1e-14.  That early stop is not always safe: on a
// domain-decomposition tree with mirror-symmetric clusters it leaves one
// recompression's basis off by about 1e-12 relative, which a run to a sweep
// without rotation avoids (at about one more sweep per call).
template <int g, int RPL>
__device__ int wave_jacobi_reg(int m, int n, MV G, MV *J) {
  const int lane = lane_id();
  const int np = n + (n & 1);
  const int npairs = np / 2;
  const int gid = lane / g, gl = lane % g;
  const double tol = 4.0e-16 * (double)(m > 8 ? m : 8), tol2 = tol * tol;
  int ri[RPL], rj[RPL];
  bool rok[RPL];
#pragma unroll
  for (int k = 0; k < RPL; ++k) {
    const int i = gl + k * g;
    rok[k] = i < m;
    ri[k] = i < m ? i : m - 1;
    rj[k] = i < n ? i : n - 1;
  }
  int sweeps = 0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    int rotated = 0, big = 0;
    for (int r = 0; r < np - 1; ++r) {
      int a = 0, b = 0;
      if (gid < npairs) {
        if (gid == 0) { a = np - 1; b = r; }
        else {
          a = r + gid; if (a >= np - 1) a -= np - 1;
          b = r - gid + np - 1; if (b >= np - 1) b -= np - 1;
        }
        if (a > b) { const int tt = a; a = b; b = tt; }
      }
      const bool act = gid < npairs && b < n;
      const int ca = act ? a : 0, cb = act ? b : 0;
      double x[RPL], y[RPL];
      double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
      for (int k = 0; k < RPL; ++k) { x[k] = G(ri[k], ca); y[k] = G(ri[k], cb); }
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const double xk = rok[k] ? x[k] : 0.0, yk = rok[k] ? y[k] : 0.0;
        al = fma(xk, xk, al); be = fma(yk, yk, be); ga = fma(xk, yk, ga);
      }
      if (!act) { al = 0.0; be = 0.0; ga = 0.0; }
      group_sum3<g>(al, be, ga);
      if (act && ga != 0.0 && ga * ga > tol2 * (al * be)) {
        double c, s;
        jacobi_rotation_fast(al, be, ga, c, s);
        if (ga * ga > 1e-14 * (al * be)) big = 1;
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
          G(ri[k], ca) = c * x[k] - s * y[k];
          G(ri[k], cb) = s * x[k] + c * y[k];
        }
        if (J != nullptr) {
          const MV Jm = *J;
          double u[RPL], v[RPL];
#pragma unroll
          for (int k = 0; k < RPL; ++k) { u[k] = Jm(rj[k], ca); v[k] = Jm(rj[k], cb); }
#pragma unroll
          for (int k = 0; k < RPL; ++k) {
            Jm(rj[k], ca) = c * u[k] - s * v[k];
            Jm(rj[k], cb) = s * u[k] + c * v[k];
          }
        }
        rotated = 1;
      }
      wave_sync();
    }
    ++sweeps;
    if (__ballot(rotated) == 0 || __ballot(big) == 0) break;
  }
  return sweeps;
}

__device__ int wave_jacobi_loop(int m, int n, MV G, MV *J) {
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
    int rotated = 0, big = 0;
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
          jacobi_rotation_fast(al, be, ga, c, s);
          if (ga * ga > 1e-14 * (al * be)) big = 1;
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
    if (__ballot(rotated) == 0 || __ballot(big) == 0) break;
  }
  return sweeps;
}

__device__ int wave_jacobi(int m, int n, MV G, MV *J) {
  if (n < 2 || m < 1) return 0;
  const int npairs = (n + (n & 1)) / 2;
  int g = 16;
  while (g > 1 && npairs * g > 64) g >>= 1;
  const int rows = (J != nullptr && n > m) ? n : m;
  if (g == 16) {
    if (rows <= 16) return wave_jacobi_reg<16, 1>(m, n, G, J);
    if (rows <= 32) return wave_jacobi_reg<16, 2>(m, n, G, J);
    if (rows <= 64) return wave_jacobi_reg<16, 4>(m, n, G, J);
  } else if (g == 8) {
    if (rows <= 16) return wave_jacobi_reg<8, 2>(m, n, G, J);
    if (rows <= 32) return wave_jacobi_reg<8, 4>(m, n, G, J);
    if (rows <= 64) return wave_jacobi_reg<8, 8>(m, n, G, J);
  } else if (g == 4) {
    if (rows <= 32) return wave_jacobi_reg<4, 8>(m, n, G, J);
  }
  return wave_jacobi_loop(m, n, G, J);
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

// ------------------------------------------------ products on the matrix cores
// One wave forms an m x n product sum_l a(i, l) b(l, j), 0 <= l < k, in
// 16 x 16 tiles on the matrix cores and hands every entry to store(i, j, v).
// The operands are accessors (a(i, l), b(l, j) may compute an entry, e.g.
// of an implicitly extended coupling); they are only called with
// 0 <= i < m, 0 <= l < k, 0 <= j < n (indices past the end are clamped and
// the loaded value replaced by zero).  Per v_mfma_f64_16x16x4f64 lane l
// supplies a(i0 + l%16, k0 + l/16) and b(k0 + l/16, j0 + l%16), and result
// register r of lane l is entry (i0 + l/16 + 4r, j0 + l%16).  Four k-steps
// are loaded together before their four matrix instructions.
typedef double h2_d4 __attribute__((ext_vector_type(4)));
typedef float h2_f4 __attribute__((ext_vector_type(4)));

template <class FA, class FB, class FS>
__device__ __forceinline__ void wv_mm_f64(int m, int n, int k, FA a, FB b, FS store) {
  const int lane = lane_id();
  const int li = lane & 15, lk = lane >> 4;
  for (int i0 = 0; i0 < m; i0 += 16) {
    const int ia = i0 + li;
    const bool iok = ia < m;
    const int ic = iok ? ia : m - 1;
    for (int j0 = 0; j0 < n; j0 += 16) {
      const int jb = j0 + li;
      const bool jok = jb < n;
      const int jc = jok ? jb : n - 1;
      h2_d4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < k; k0 += 16) {
        double x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int kk = k0 + 4 * u + lk;
          const bool kok = kk < k;
          const int kc = kok ? kk : k - 1;
          const double av = a(ic, kc), bv = b(kc, jc);
          x[u] = (iok && kok) ? av : 0.0;
          y[u] = (jok && kok) ? bv : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x[u], y[u], acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + lk + 4 * r;
        if (i < m && jok) store(i, jb, acc[r]);
      }
    }
  }
}

// The same product with the operands rounded to float and accumulated in
// float (v_mfma_f32_16x16x4f32: same operand layout, result register r of
// lane l is entry (i0 + 4(l/16) + r, j0 + l%16)); store receives the float
// result widened to double.  The mixed-precision form of the coupling and
// transfer products.
template <class FA, class FB, class FS>
__device__ __forceinline__ void wv_mm_f32(int m, int n, int k, FA a, FB b, FS store) {
  const int lane = lane_id();
  const int li = lane & 15, lk = lane >> 4;
  for (int i0 = 0; i0 < m; i0 += 16) {
    const int ia = i0 + li;
    const bool iok = ia < m;
    const int ic = iok ? ia : m - 1;
    for (int j0 = 0; j0 < n; j0 += 16) {
      const int jb = j0 + li;
      const bool jok = jb < n;
      const int jc = jok ? jb : n - 1;
      h2_f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
      for (int k0 = 0; k0 < k; k0 += 16) {
        float x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int kk = k0 + 4 * u + lk;
          const bool kok = kk < k;
          const int kc = kok ? kk : k - 1;
          const double av = a(ic, kc), bv = b(kc, jc);
          x[u] = (iok && kok) ? (float)av : 0.0f;
          y[u] = (jok && kok) ? (float)bv : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u], y[u], acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + 4 * lk + r;
        if (i < m && jok) store(i, jb, (double)acc[r]);
      }
    }
  }
}

// Precision switch: f32 selects the float form.
template <class FA, class FB, class FS>
__device__ __forceinline__ void wv_mm(bool f32, int m, int n, int k, FA a, FB b, FS store) {
  if (f32) wv_mm_f32(m, n, k, a, b, store);
  else wv_mm_f64(m, n, k, a, b, store);
}

// C (m x n) = alpha * A (m x k) * B (k x n) + beta * C (no aliasing), on
// the matrix cores (float operands and accumulation if f32).
__device__ void wv_gemm(int m, int n, int k, double alpha, MV A, MV B, double beta, MV C, bool f32 = false) {
  if (m > 0 && n > 0) {
    auto st = [&](int i, int j, double v) { C(i, j) = (beta == 0.0 ? 0.0 : beta * C(i, j)) + alpha * v; };
    if (k > 0) wv_mm(f32, m, n, k, [&](int i, int l) { return A(i, l); }, [&](int l, int j) { return B(l, j); }, st);
    else {
      for (int q = lane_id(); q < m * n; q += 64) st(q % m, q / m, 0.0);
    }
  }
  wave_sync();
}

// Trailing update of Householder step j (helper of wv_qr).  The lanes form
// column groups of RG = 2^LG adjacent lanes: lane (g, r) handles the columns
// c = j+1+g, j+1+g+64/RG, ... on the rows j+1+r (mod RG), in chunks of RPL
// rows whose loads are issued together (ONE: all rows fit in one chunk and
// stay in registers between the dot product and the update).  Row indices
// past the end are clamped to the lane's own first row of the chunk: such
// entries contribute zero to the dot products and are stored again with the
// value just computed for that row, so loads and stores need no branches and
// a duplicate store never sees an already updated entry.  Returns, in every
// lane, the squared norm of column j+1 below its diagonal after the update.
template <int LG, int RPL, bool ONE>
__device__ __forceinline__ double wv_qr_step(int m, int n, int j, MV A, double t, double scale) {
  constexpr int RG = 1 << LG, CG = 64 >> LG;
  const int lane = lane_id();
  const int g = lane >> LG, r = lane & (RG - 1);
  double snext = 0.0;
  for (int c = j + 1 + g; c < n; c += CG) {
    const double ajc = A(j, c);
    double q = 0.0, coef;
    if (ONE) {
      const int i0 = j + 1 + r < m ? j + 1 + r : j + 1;
      double vj[RPL], vc[RPL];
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int i = j + 1 + r + k * RG, ic = i < m ? i : i0;
        vj[k] = A(ic, j);
        vc[k] = A(ic, c);
      }
      double p = 0.0;
#pragma unroll
      for (int k = 0; k < RPL; ++k) p = fma(j + 1 + r + k * RG < m ? vj[k] : 0.0, vc[k], p);
      p = group_sum_t<RG>(p);
      coef = t * fma(scale, p, ajc);
      const double f = coef * scale;
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int i = j + 1 + r + k * RG, ic = i < m ? i : i0;
        const double a = fma(-f, vj[k], vc[k]);
        A(ic, c) = a;
        q = fma(i < m && i > j + 1 ? a : 0.0, a, q);   // rows below the next diagonal entry
      }
    } else {
      double p = 0.0;
      for (int i0 = j + 1 + r; i0 < m; i0 += RG * RPL) {
        double vj[RPL], vc[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
          const int i = i0 + k * RG, ic = i < m ? i : i0;
          vj[k] = A(ic, j);
          vc[k] = A(ic, c);
        }
#pragma unroll
        for (int k = 0; k < RPL; ++k) p = fma(i0 + k * RG < m ? vj[k] : 0.0, vc[k], p);
      }
      p = group_sum_t<RG>(p);
      coef = t * fma(scale, p, ajc);
      const double f = coef * scale;
      for (int i0 = j + 1 + r; i0 < m; i0 += RG * RPL) {
        double vj[RPL], vc[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
          const int i = i0 + k * RG, ic = i < m ? i : i0;
          vj[k] = A(ic, j);
          vc[k] = A(ic, c);
        }
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
          const int i = i0 + k * RG, ic = i < m ? i : i0;
          const double a = fma(-f, vj[k], vc[k]);
          A(ic, c) = a;
          q = fma(i < m && i > j + 1 ? a : 0.0, a, q);
        }
      }
    }
    if (r == 0) A(j, c) = ajc - coef;
    if (c == j + 1) snext = q;
  }
  // the group of column j+1 is g = 0 (lanes 0 .. RG-1)
  snext = group_sum_t<RG>(snext);
  return bcast_lane0(snext);
}

template <int LG>
__device__ __forceinline__ double wv_qr_step_rows(int m, int n, int j, MV A, double t, double scale) {
  constexpr int RG = 1 << LG;
  const int mt = m - j - 1;
  if (mt <= 2 * RG) return wv_qr_step<LG, 2, true>(m, n, j, A, t, scale);
  if (mt <= 4 * RG) return wv_qr_step<LG, 4, true>(m, n, j, A, t, scale);
  if (mt <= 8 * RG) return wv_qr_step<LG, 8, true>(m, n, j, A, t, scale);
  return wv_qr_step<LG, 8, false>(m, n, j, A, t, scale);
}

// Householder QR in place, one wave: R in the upper triangle; below it the
// reflectors v (unit leading entry implied) and tau[j] when tau != nullptr,
// otherwise unspecified values.  The squared norm that step j+1 needs is
// accumulated by the trailing update of step j.  The reciprocals and the
// square root use the hardware approximations refined by Newton steps.
__device__ void wv_qr(int m, int n, MV A, double *tau) {
  const int lane = lane_id();
  const int kmax = m < n ? m : n;
  double s = 0.0;
  if (kmax > 0) {
    for (int i = 1 + lane; i < m; i += 64) { const double v = A(i, 0); s = fma(v, v, s); }
    s = wave_sum64(s);
  }
  for (int j = 0; j < kmax; ++j) {
    const double alpha = A(j, j);
    double t = 0.0, beta = alpha, scale = 0.0;
    if (s > 0.0) {
      const double nrm = sqrt_nr(fma(alpha, alpha, s));
      beta = alpha >= 0.0 ? -nrm : nrm;
      const double rb = rcp_nr(beta), rd = rcp_nr(alpha - beta);
      t = (beta - alpha) * rb;
      scale = rd;
    }
    const int nt = n - j - 1, mt = m - j - 1;
    double snext = 0.0;
    if (t != 0.0) {
      if (nt <= 4 && mt >= 48) snext = wv_qr_step_rows<4>(m, n, j, A, t, scale);
      else if (nt <= 8 && mt >= 24) snext = wv_qr_step_rows<3>(m, n, j, A, t, scale);
      else snext = wv_qr_step_rows<2>(m, n, j, A, t, scale);
      if (tau != nullptr) {
        for (int i = j + 1 + lane; i < m; i += 64) A(i, j) *= scale;
      }
      if (lane == 0) A(j, j) = beta;
      wave_sync();
    } else {
      for (int i = j + 1 + lane; i < m; i += 64) A(i, j) = 0.0;
      wave_sync();
      for (int i = j + 2 + lane; i < m && j + 1 < n; i += 64) { const double v = A(i, j + 1); snext = fma(v, v, snext); }
      snext = wave_sum64(snext);
    }
    if (tau != nullptr && lane == 0) tau[j] = t;
    s = snext;
  }
  wave_sync();
}

// Z <- H_j Z for the Householder reflector H_j = I - tau v v^* stored by
// wv_qr in column j of A (v_j = 1, v_i = A(i, j) below), applied to the
// columns 0..nz-1 of Z (m rows).  Same lane layout and clamping as
// wv_qr_step.
template <int LG, int RPL, bool ONE>
__device__ __forceinline__ void wv_refl_apply(int m, int j, MV A, double tau, MV Z, int nz) {
  constexpr int RG = 1 << LG, CG = 64 >> LG;
  const int lane = lane_id();
  const int g = lane >> LG, r = lane & (RG - 1);
  for (int c = g; c < nz; c += CG) {
    const double zjc = Z(j, c);
    double p = 0.0;
    if (ONE) {
      const int i0 = j + 1 + r < m ? j + 1 + r : j + 1;
      double v[RPL], z[RPL];
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int i = j + 1 + r + k * RG, ic = i < m ? i : i0;
        v[k] = A(ic, j);
        z[k] = Z(ic, c);
      }
#pragma unroll
      for (int k = 0; k < RPL; ++k) p = fma(j + 1 + r + k * RG < m ? v[k] : 0.0, z[k], p);
      p = group_sum_t<RG>(p);
      const double w = tau * (zjc + p);
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int i = j + 1 + r + k * RG, ic = i < m ? i : i0;
        Z(ic, c) = fma(-w, v[k], z[k]);
      }
      if (r == 0) Z(j, c) = zjc - w;
    } else {
      for (int i0 = j + 1 + r; i0 < m; i0 += RG * RPL) {
        double v[RPL], z[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
          const int i = i0 + k * RG, ic = i < m ? i : i0;
          v[k] = A(ic, j);
          z[k] = Z(ic, c);
        }
#pragma unroll
        for (int k = 0; k < RPL; ++k) p = fma(i0 + k * RG < m ? v[k] : 0.0, z[k], p);
      }
      p = group_sum_t<RG>(p);
      const double w = tau * (zjc + p);
      for (int i0 = j + 1 + r; i0 < m; i0 += RG * RPL) {
        double v[RPL], z[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
          const int i = i0 + k * RG, ic = i < m ? i : i0;
          v[k] = A(ic, j);
          z[k] = Z(ic, c);
        }
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
          const int i = i0 + k * RG, ic = i < m ? i : i0;
          Z(ic, c) = fma(-w, v[k], z[k]);
        }
      }
      if (r == 0) Z(j, c) = zjc - w;
    }
  }
}

// Z <- Q Z with Q = H_0 H_1 ... H_{n-1} from wv_qr(m, n, A, tau) (m rows,
// nz columns of Z), one wave.
__device__ void wv_apply_q(int m, int n, MV A, const double *tau, MV Z, int nz) {
  const int kmax = m < n ? m : n;
  for (int j = kmax - 1; j >= 0; --j) {
    const double t = tau[j];
    if (t != 0.0 && nz > 0) {
      const int mt = m - j - 1;
      if (mt <= 8) wv_refl_apply<2, 2, true>(m, j, A, t, Z, nz);
      else if (mt <= 16) wv_refl_apply<2, 4, true>(m, j, A, t, Z, nz);
      else if (mt <= 32) wv_refl_apply<2, 8, true>(m, j, A, t, Z, nz);
      else wv_refl_apply<2, 8, false>(m, j, A, t, Z, nz);
    }
    wave_sync();
  }
}

// Column norms of G (m x n) into sig, groups of 2^LG lanes per column.
template <int LG>
__device__ __forceinline__ void wv_colnorms(int m, int n, MV G, double *sig) {
  constexpr int g = 1 << LG;
  const int lane = lane_id(), gl = lane & (g - 1);
  for (int c0 = 0; c0 < n; c0 += 64 >> LG) {
    const int c = c0 + (lane >> LG);
    double s = 0.0;
    if (c < n) {
      for (int i = gl; i < m; i += g) { const double x = G(i, c); s = fma(x, x, s); }
    }
    s = group_sum_t<g>(s);
    if (c < n && gl == 0) sig[c] = sqrt(s);
  }
}

// Column norms and descending ranking, wave level.  The norms use groups of
// g lanes per column (rows split over the group, DPP reduction).
__device__ void wv_colnorms_sorted(int m, int n, MV G, double *sig, int *ord) {
  const int lane = lane_id();
  if (n <= 8) wv_colnorms<3>(m, n, G, sig);
  else if (n <= 16) wv_colnorms<2>(m, n, G, sig);
  else if (n <= 32) wv_colnorms<1>(m, n, G, sig);
  else wv_colnorms<0>(m, n, G, sig);
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

// Triangular solve by one wave, lane i holding row i of the triangular
// matrix T in row[] (as loaded by wave_load_tri): forward substitution for
// lower T (forward = true) or backward substitution for upper T; unit: the
// diagonal is taken as 1 and not read.
template <int NMAX>
__device__ __forceinline__ double wave_tri_solve_ex(int n, const double (&row)[NMAX], bool forward, bool unit,
                                                    double b) {
  const int lane = lane_id();
  if (forward) {
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
      if (j < n) {
        const double bj = __shfl(b, j, 64);
        const double xj = unit ? bj : bj / __shfl(row[j], j, 64);
        if (lane == j) b = xj;
        else if (lane > j) b = fma(-row[j], xj, b);
      }
    }
  } else {
#pragma unroll
    for (int j = NMAX - 1; j >= 0; --j) {
      if (j < n) {
        const double bj = __shfl(b, j, 64);
        const double xj = unit ? bj : bj / __shfl(row[j], j, 64);
        if (lane == j) b = xj;
        else if (lane < j) b = fma(-row[j], xj, b);
      }
    }
  }
  return b;
}

// B (n x m) <- T^{-1} B, n <= LS, one wave per column of B.  T is the lower
// (forward = true) or upper triangle of A (load_trans = 0) or of A^T
// (load_trans = 1); unit: unit diagonal.  The LR factor of a leaf holds the
// unit lower L below and R on and above the diagonal:
//   L^{-1} B: load_trans 0, forward, unit;   R^{-1} B: load_trans 0, backward;
//   R^{-T} B: load_trans 1, forward.
__device__ void wg_trsv_ex(int n, int m, MV A, MV B, int load_trans, bool forward, bool unit) {
  double row[LS];
  wave_load_tri<LS>(n, A, load_trans, row);
  const int lane = lane_id();
  for (int c = wave_id(); c < m; c += num_waves()) {
    double b = lane < n ? B(lane, c) : 0.0;
    b = wave_tri_solve_ex<LS>(n, row, forward, unit, b);
    if (lane < n) B(lane, c) = b;
  }
  __syncthreads();
}

// Gaussian elimination without pivoting of A (n x n) in place: A <- (L - I)
// + R with L unit lower and R upper triangular.  Returns 0, or j + 1 for the
// first zero pivot A(j, j) (that pivot is then replaced by 1 so that the
// remaining steps stay finite).
__device__ int wg_getrf_nopiv(int n, MV A, int *iflag) {
  if (threadIdx.x == 0) *iflag = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double piv = A(j, j);
    __syncthreads();
    if (piv == 0.0) {
      if (threadIdx.x == 0) { if (*iflag == 0) *iflag = j + 1; A(j, j) = 1.0; }
    }
    const double d = piv == 0.0 ? 1.0 : piv;
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) A(i, j) /= d;
    __syncthreads();
    const int rem = n - j - 1;
    for (int idx = threadIdx.x; idx < rem * rem; idx += blockDim.x) {
      const int i = j + 1 + idx % rem, c = j + 1 + idx / rem;
      A(i, c) = fma(-A(i, j), A(j, c), A(i, c));
    }
    __syncthreads();
  }
  const int r = *iflag;
  __syncthreads();
  return r;
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


// A (n x n, n <= LS) <- L^{-1} for the lower triangular L held in A; the
// strict upper triangle of the result is exactly zero.  Column c of the
// inverse solves L x = e_c; one wave per column, L staged in registers by
// every wave before any column is written.
__device__ void wg_trtri_lower(int n, MV A) {
  double row[LS];
  wave_load_tri<LS>(n, A, 0, row);
  __syncthreads();
  const int lane = lane_id();
  for (int c = wave_id(); c < n; c += num_waves()) {
    double b = lane == c ? 1.0 : 0.0;
    b = wave_tri_solve<LS>(n, row, 0, b);
    if (lane < n) A(lane, c) = b;
  }
  __syncthreads();
}

// B (n x m) <- L B (trans = 0) or L^T B (trans = 1) for the lower triangle
// of L (n <= LS; entries above the diagonal are ignored), in place; one wave
// per column of B.
__device__ void wg_trmv_lower(int n, int m, MV L, MV B, int trans) {
  double row[LS];
  wave_load_tri<LS>(n, L, trans, row);
  const int lane = lane_id();
  for (int c = wave_id(); c < m; c += num_waves()) {
    const double x = lane < n ? B(lane, c) : 0.0;
    double acc = 0.0;
#pragma unroll
    for (int l = 0; l < LS; ++l) {
      const double xl = __shfl(x, l, 64);
      const bool in_tri = trans ? (l >= lane) : (l <= lane);
      if (l < n && in_tri) acc = fma(row[l], xl, acc);
    }
    if (lane < n) B(lane, c) = acc;
  }
  __syncthreads();
}

}  // namespace h2
