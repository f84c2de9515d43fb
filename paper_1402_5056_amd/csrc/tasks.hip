// Device tasks of the H^2 arithmetic and the task interpreter.
//
// The host turns every operation (local low-rank update, product recursion,
// block substitution, Cholesky) into a static list of tasks that depends only
// on the trees.  Ranks and all numerical data live on the device; a task reads
// the current ranks when it runs.  One workgroup executes a list in order, so
// the long chain of small dependent updates costs no kernel launches.
#include <hip/hip_runtime.h>
#include "common.h"
#include "dense.h"

namespace h2 {

constexpr int W0R = 128;   // rows of the stack work area in LDS

struct Lds {
  double *W0;   // W0R x KM, col-major, ld W0R
  double *W1;   // KM x KM, ld KM
  double *W2;   // KM x KM, ld KM
  double *red;  // NT
  double *sig;  // KM
  double *tau;  // 2 * KM
  int *iw;      // 4 * KM ints
};
constexpr size_t LDS_DOUBLES = (size_t)W0R * KM + 2 * KM * KM + NT + KM + 2 * KM + 2 * KM;

__device__ __forceinline__ Lds lds_layout(double *base) {
  Lds L;
  L.W0 = base;
  L.W1 = L.W0 + W0R * KM;
  L.W2 = L.W1 + KM * KM;
  L.red = L.W2 + KM * KM;
  L.sig = L.red + NT;
  L.tau = L.sig + KM;
  L.iw = reinterpret_cast<int *>(L.tau + 2 * KM);
  return L;
}

// ------------------------------------------------------------ tree helpers
__device__ __forceinline__ bool is_leaf(const DevEnv &e, int c) { return e.son0[c] < 0; }
__device__ __forceinline__ bool in_sub(const DevEnv &e, int root, int c) {
  const int a = e.offset[root], b = a + e.size[root];
  const int x = e.offset[c];
  return x >= a && x + e.size[c] <= b && e.level[c] >= e.level[root];
}
__device__ __forceinline__ int dlo(const DevEnv &e, int c, int lv) { return e.desc_lo[c * e.nlev + lv]; }
__device__ __forceinline__ int dhi(const DevEnv &e, int c, int lv) { return e.desc_hi[c * e.nlev + lv]; }

__device__ __forceinline__ MV leafslot(const DevEnv &e, int side, int c) {
  return mv_col(e.leaf[side] + (long)c * LS * KC, LS);
}
__device__ __forceinline__ MV Eslot(const DevEnv &e, int side, int c) {
  return mv_col(e.E[side] + (long)c * KC * KC, KC);
}
__device__ __forceinline__ MV rhoslot(const DevEnv &e, int side, int c) {
  return mv_col(e.rho[side] + (long)c * KC * KC, KC);
}
__device__ __forceinline__ MV Sslot(const DevEnv &e, int b) {
  return mv_col(e.S + (long)e.bslot[b] * KC * KC, KC);
}
__device__ __forceinline__ MV Nslot(const DevEnv &e, int b) {
  return mv_col(e.N + (long)e.bslot[b] * LS * LS, LS);
}
__device__ __forceinline__ MV wslot(double *base, int c) { return mv_col(base + (long)c * KM * KM, KM); }
__device__ __forceinline__ MV xhslot(double *base, int c) { return mv_row(base + (long)c * KC * BC, BC); }
__device__ __forceinline__ MV bufrows(const DevEnv &e, int bi, int c) {
  return mv_row(e.buf[bi] + (long)e.offset[c] * BC, BC);
}
__device__ __forceinline__ MV bufrow0(const DevEnv &e, int bi, int row) {
  return mv_row(e.buf[bi] + (long)row * BC, BC);
}

__device__ __forceinline__ void set_error(const DevEnv &e, int code, int info) {
  if (threadIdx.x == 0 && e.err[0] == 0) { e.err[1] = info; e.err[0] = code; }
  __syncthreads();
}

__device__ __forceinline__ double trunc_tau(const DevEnv &e, double smax) {
  if (e.mode == 0) return e.eps;
  if (e.mode == 1) return e.eps * smax;
  return 0.0;
}

// ------------------------------------------------------- flop accounting
// Algorithmic flops of the dense steps (conventions: product 2mnk,
// Householder R-factor 2mn^2 - 2n^3/3 for m >= n, SVD with left vectors
// 4ab^2 + 8b^3 with a = max, b = min).  Counted by thread 0 only.
__device__ __forceinline__ double fl_gemm(double m, double n, double k) { return 2.0 * m * n * k; }
__device__ __forceinline__ double fl_qr(double m, double n) {
  return m >= n ? 2.0 * m * n * n - 2.0 * n * n * n / 3.0 : 2.0 * n * m * m - 2.0 * m * m * m / 3.0;
}
__device__ __forceinline__ double fl_svd(double m, double n) {
  const double a = m > n ? m : n, b = m > n ? n : m;
  return 4.0 * a * b * b + 8.0 * b * b * b;
}
__device__ __forceinline__ void count(const DevEnv &e, double f) {
  if (threadIdx.x == 0 && e.flops) e.flops[0] += f;
}

// ======================================================= low-rank update
struct Upd {
  int r0[2];   // t0, s0
  int buf[2];  // X, Y buffers
  int kp;
};

// R-factor of the (possibly extended) basis of cluster c.
__device__ __forceinline__ MV rho_of(const DevEnv &e, const Upd &u, int side, int c, int &m) {
  if (in_sub(e, u.r0[side], c)) { m = e.wrho_m[side][c]; return wslot(e.wrho[side], c); }
  m = e.rho_m[side][c];
  return rhoslot(e, side, c);
}

// Extended coupling S~_b (K_t x K_s) into dst (Section 5, three rules).
__device__ void load_stilde(const DevEnv &e, const Upd &u, int b, MV dst, int &Kt, int &Ks) {
  const int t = e.brow[b], s = e.bcol[b];
  const int kt = e.k[0][t], ks = e.k[1][s];
  const bool tin = in_sub(e, u.r0[0], t), sin = in_sub(e, u.r0[1], s);
  Kt = kt + (tin ? u.kp : 0);
  Ks = ks + (sin ? u.kp : 0);
  MV S = Sslot(e, b);
  const int tot = Kt * Ks;
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int i = idx % Kt, j = idx / Kt;
    double v;
    if (i < kt && j < ks) v = S(i, j);
    else v = (tin && sin && i >= kt && j >= ks && (i - kt) == (j - ks)) ? 1.0 : 0.0;
    dst(i, j) = v;
  }
  __syncthreads();
}

// Block scale omega_b = 1/||R_{V,t} S~_b R_{W,s}^*||_F; leaves S~_b in L.W2.
__device__ double block_scale(const DevEnv &e, const Upd &u, const Lds &L, int b, int &Kt, int &Ks) {
  MV St = mv_col(L.W2, KM);
  load_stilde(e, u, b, St, Kt, Ks);
  if (e.mode != 0) return 1.0;
  int mt, ms;
  MV Rt = rho_of(e, u, 0, e.brow[b], mt);
  MV Rs = rho_of(e, u, 1, e.bcol[b], ms);
  MV P = mv_col(L.W1, KM);
  wg_gemm(mt, Ks, Kt, 1.0, Rt, St, 0.0, P);
  double acc = 0.0;
  const int tot = mt * ms;
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int i = idx % mt, j = idx / mt;
    double s = 0.0;
    for (int l = 0; l < Ks; ++l) s = fma(P(i, l), Rs(j, l), s);
    acc = fma(s, s, acc);
  }
  const double f2 = wg_sum(acc, L.red);
  return f2 > 0.0 ? 1.0 / sqrt(f2) : 0.0;
}

// Compress the stack rows [0, m) x K of W0 to its R-factor; returns new m.
__device__ int stack_compress(const Lds &L, int m, int K) {
  MV A = mv_col(L.W0, W0R);
  wg_qr(m, K, A, nullptr, L.red);
  wg_clean_r(m, K, A);
  return m < K ? m : K;
}

// Weight matrix B~_t (Section 4, recursion for the weights; all blocks of
// row(t) as required by Section 5).  insub: t lies in the updated subtree.
__device__ void build_weight(const DevEnv &e, const Upd &u, const Lds &L, int side, int t, bool insub) {
  const int kt = e.k[side][t];
  const int Kt = kt + (insub ? u.kp : 0);
  MV A = mv_col(L.W0, W0R);
  int m = 0, mrows = 0;
  const int *ptr = side == 0 ? e.rowptr : e.colptr;
  const int *idx = side == 0 ? e.rowidx : e.colidx;
  for (int p = ptr[t]; p < ptr[t + 1]; ++p) {
    const int b = idx[p];
    int Kbt, Kbs;
    const double w = block_scale(e, u, L, b, Kbt, Kbs);   // S~ in W2
    if (w == 0.0) continue;
    const int other = side == 0 ? e.bcol[b] : e.brow[b];
    int mo;
    MV Ro = rho_of(e, u, 1 - side, other, mo);
    if (mo == 0) continue;
    if (m + mo > W0R) m = stack_compress(L, m, Kt);
    MV St = mv_col(L.W2, KM);
    // side 0: w * R_{W,s} S~^T (mo x K_t); side 1: w * R_{V,t} S~ (mo x K_s)
    MV B = side == 0 ? mv_t(St) : St;
    const int Ko = side == 0 ? Kbs : Kbt;
    wg_gemm(mo, Kt, Ko, w, Ro, B, 0.0, mv_at(A, m, 0));
    if (e.mode == 0) {
      int mt, ms;
      (void)rho_of(e, u, 0, e.brow[b], mt);
      (void)rho_of(e, u, 1, e.bcol[b], ms);
      count(e, fl_gemm(mt, Kbs, Kbt) + fl_gemm(mt, ms, Kbs));
    }
    count(e, fl_gemm(mo, Kt, Ko));
    mrows += mo;
    m += mo;
  }
  const int par = e.parent[t];
  if (par >= 0) {
    const bool pin = in_sub(e, u.r0[side], par);
    const int kpar = e.k[side][par];
    const int Kp = kpar + (pin ? u.kp : 0);
    const int mp = e.wB_m[side][par];
    if (mp > 0) {
      if (m + mp > W0R) m = stack_compress(L, m, Kt);
      MV Bp = wslot(e.wB[side], par);
      MV Et = Eslot(e, side, t);
      const bool root_of_sub = insub && t == u.r0[side];
      MV D = mv_at(A, m, 0);
      const int tot = mp * Kt;
      for (int q = threadIdx.x; q < tot; q += blockDim.x) {
        const int i = q % mp, j = q / mp;
        double s = 0.0;
        if (j < kt) {
          for (int l = 0; l < kpar; ++l) s = fma(Bp(i, l), Et(j, l), s);
        } else if (!root_of_sub) {
          s = Bp(i, kpar + (j - kt));   // identity part of diag(E_t, I)
        }
        D(i, j) = s;
      }
      __syncthreads();
      count(e, fl_gemm(mp, kt, kpar));
      mrows += mp;
      m += mp;
    }
  }
  count(e, fl_qr(mrows, Kt));
  MV W = wslot(e.wB[side], t);
  if (m > 0) {
    wg_qr(m, Kt, A, nullptr, L.red);
    const int mr = m < Kt ? m : Kt;
    wg_extract_r(m, Kt, A, W);
    if (threadIdx.x == 0) e.wB_m[side][t] = mr;
  } else {
    if (threadIdx.x == 0) e.wB_m[side][t] = 0;
  }
  __syncthreads();
}

// Truncated SVD of M = L.W2 (m x n): left singular vectors of the kept part
// into Q (m x r, W0), returns r (or -1 past the rank cap).  For n <= m the
// columns of M are orthogonalised (left vectors = normalised columns); for
// n > m the columns of M^* are, and the accumulated rotations are the left
// singular vectors of M.
__device__ int recompress_svd(const DevEnv &e, const Lds &L, int m, int n, MV Q) {
  MV M = mv_col(L.W2, KM);
  int *ord = L.iw + KM;
  const bool trans = n > m;
  const int nG = trans ? m : n;
  int sweeps;
  MV J = mv_at(mv_col(L.W0, W0R), 64, 0);      // rows 64.. of W0 (m x m)
  if (!trans) {
    sweeps = wg_jacobi(m, n, M, nullptr, L.iw);
    wg_colnorms_sorted(m, n, M, L.sig, ord);
  } else {
    for (int q = threadIdx.x; q < m * m; q += blockDim.x) J(q % m, q / m) = (q % m == q / m) ? 1.0 : 0.0;
    __syncthreads();
    MV Mt = mv_t(M);
    sweeps = wg_jacobi(n, m, Mt, &J, L.iw);
    wg_colnorms_sorted(n, m, Mt, L.sig, ord);
  }
  if (e.prof && threadIdx.x == 0) {
    e.prof[PROF_STAGE + 12] += sweeps;
    e.prof[PROF_STAGE + 13] += 1;
    e.prof[PROF_STAGE + 14] += nG;
  }
  count(e, fl_svd(m, n));
  const double tau = trunc_tau(e, nG > 0 ? L.sig[ord[0]] : 0.0);
  int r = 0;
  for (int j = 0; j < nG; ++j) r += L.sig[ord[j]] > tau ? 1 : 0;
  if (r > e.rank_cap) return -1;
  for (int q = threadIdx.x; q < m * r; q += blockDim.x) {
    const int i = q % m, j = q / m;
    const int c = ord[j];
    Q(i, j) = trans ? J(i, c) : M(i, c) / L.sig[c];
  }
  __syncthreads();
  return r;
}

__device__ __forceinline__ void prof_stage(const DevEnv &e, int stage, unsigned long long &t) {
  if (e.prof && threadIdx.x == 0) {
    const unsigned long long now = wall_clock64();
    e.prof[PROF_STAGE + stage] += now - t;
    t = now;
  }
}

__device__ void task_addlr(const DevEnv &e, const Lds &L, int b0, int bx, int by) {
  unsigned long long tstage = wall_clock64();
  Upd u;
  u.r0[0] = e.brow[b0];
  u.r0[1] = e.bcol[b0];
  u.buf[0] = bx;
  u.buf[1] = by;
  u.kp = e.bcols[bx];
  if (u.kp <= 0) return;
  if (u.kp > KPMAX || e.bcols[by] != u.kp) { set_error(e, E_ARG, b0); return; }
  // --- skip an identically zero update
  {
    int nz = 0;
    for (int side = 0; side < 2; ++side) {
      int any = 0;
      MV F = bufrows(e, u.buf[side], u.r0[side]);
      const int rows = e.size[u.r0[side]];
      for (int q = threadIdx.x; q < rows * u.kp; q += blockDim.x)
        if (F(q / u.kp, q % u.kp) != 0.0) any = 1;
      nz += wg_or(any, L.iw);
    }
    if (nz < 2) return;
  }
  prof_stage(e, 0, tstage);
  const int kp = u.kp;
  // --- step 1: R-factors of the extended bases, bottom-up
  for (int side = 0; side < 2; ++side) {
    const int root = u.r0[side];
    for (int lv = e.nlev - 1; lv >= e.level[root]; --lv) {
      const int lo = dlo(e, root, lv), hi = dhi(e, root, lv);
      for (int c = lo; c < hi; ++c) {
        const int kc = e.k[side][c];
        const int K = kc + kp;
        MV A = mv_col(L.W0, W0R);
        int m;
        if (is_leaf(e, c)) {
          m = e.size[c];
          MV V = leafslot(e, side, c);
          MV F = bufrows(e, u.buf[side], c);
          for (int q = threadIdx.x; q < m * K; q += blockDim.x) {
            const int i = q % m, j = q / m;
            A(i, j) = j < kc ? V(i, j) : F(i, j - kc);
          }
          __syncthreads();
        } else {
          m = 0;
          for (int sn = 0; sn < 2; ++sn) {
            const int ch = sn == 0 ? e.son0[c] : e.son1[c];
            const int mc = e.wrho_m[side][ch];
            const int kch = e.k[side][ch];
            MV Rc = wslot(e.wrho[side], ch);
            MV Ec = Eslot(e, side, ch);
            MV D = mv_at(A, m, 0);
            for (int q = threadIdx.x; q < mc * K; q += blockDim.x) {
              const int i = q % mc, j = q / mc;
              double s = 0.0;
              if (j < kc) { for (int l = 0; l < kch; ++l) s = fma(Rc(i, l), Ec(l, j), s); }
              else s = Rc(i, kch + (j - kc));
              D(i, j) = s;
            }
            __syncthreads();
            m += mc;
          }
        }
        wg_qr(m, K, A, nullptr, L.red);
        count(e, fl_qr(m, K) + (is_leaf(e, c) ? 0.0 : fl_gemm(m, kc, e.k[side][e.son0[c]])));
        wg_extract_r(m, K, A, wslot(e.wrho[side], c));
        if (threadIdx.x == 0) e.wrho_m[side][c] = m < K ? m : K;
        __syncthreads();
      }
    }
  }
  prof_stage(e, 1, tstage);
  // --- steps 2/3: weights along pred(t0) \ {t0}, then through the subtree
  for (int side = 0; side < 2; ++side) {
    const int root = u.r0[side];
    int *path = L.iw + 2 * KM;   // up to KM entries
    int np = 0;
    if (threadIdx.x == 0) {
      int c = e.parent[root];
      while (c >= 0) { path[np++] = c; c = e.parent[c]; }
      L.iw[3 * KM + 63] = np;
    }
    __syncthreads();
    np = L.iw[3 * KM + 63];
    __syncthreads();
    for (int q = np - 1; q >= 0; --q) build_weight(e, u, L, side, path[q], false);
    prof_stage(e, 2, tstage);
    for (int lv = e.level[root]; lv < e.nlev; ++lv) {
      const int lo = dlo(e, root, lv), hi = dhi(e, root, lv);
      for (int c = lo; c < hi; ++c) build_weight(e, u, L, side, c, true);
    }
    prof_stage(e, 3, tstage);
  }
  // --- step 4: nested recompression, bottom-up
  for (int side = 0; side < 2; ++side) {
    const int root = u.r0[side];
    for (int lv = e.nlev - 1; lv >= e.level[root]; --lv) {
      const int lo = dlo(e, root, lv), hi = dhi(e, root, lv);
      for (int c = lo; c < hi; ++c) {
        const int kc = e.k[side][c];
        const int K = kc + kp;
        MV Vt = mv_col(L.W1, KM);
        int mr;
        int r1 = 0;
        if (is_leaf(e, c)) {
          mr = e.size[c];
          MV V = leafslot(e, side, c);
          MV F = bufrows(e, u.buf[side], c);
          for (int q = threadIdx.x; q < mr * K; q += blockDim.x) {
            const int i = q % mr, j = q / mr;
            Vt(i, j) = j < kc ? V(i, j) : F(i, j - kc);
          }
          __syncthreads();
        } else {
          mr = 0;
          for (int sn = 0; sn < 2; ++sn) {
            const int ch = sn == 0 ? e.son0[c] : e.son1[c];
            const int rc = e.wnewk[side][ch];
            const int kch = e.k[side][ch];
            MV Rc = wslot(e.wR[side], ch);
            MV Ec = Eslot(e, side, ch);
            MV D = mv_at(Vt, mr, 0);
            for (int q = threadIdx.x; q < rc * K; q += blockDim.x) {
              const int i = q % rc, j = q / rc;
              double s = 0.0;
              if (j < kc) { for (int l = 0; l < kch; ++l) s = fma(Rc(i, l), Ec(l, j), s); }
              else s = Rc(i, kch + (j - kc));
              D(i, j) = s;
            }
            __syncthreads();
            if (sn == 0) r1 = rc;
            mr += rc;
          }
        }
        const int mB = e.wB_m[side][c];
        int r = 0;
        MV Q = mv_col(L.W0, W0R);
        if (!is_leaf(e, c)) count(e, fl_gemm(mr, kc, e.k[side][e.son0[c]]));
        if (mr > 0 && mB > 0) {
          MV M = mv_col(L.W2, KM);
          wg_gemm(mr, mB, K, 1.0, Vt, mv_t(wslot(e.wB[side], c)), 0.0, M);
          count(e, fl_gemm(mr, mB, K));
          unsigned long long tsvd = wall_clock64();
          r = recompress_svd(e, L, mr, mB, Q);
          if (e.prof && threadIdx.x == 0) e.prof[PROF_STAGE + 11] += wall_clock64() - tsvd;
          if (r < 0) { set_error(e, E_RANK_CAP, c); return; }
        }
        // basis change R_c = Q^* V~_c (r x K)
        wg_gemm(r, K, mr, 1.0, mv_t(Q), Vt, 0.0, wslot(e.wR[side], c));
        count(e, fl_gemm(r, K, mr));
        if (threadIdx.x == 0) e.wnewk[side][c] = r;
        if (is_leaf(e, c)) {
          wg_copy(mr, r, Q, leafslot(e, side, c));
        } else {
          const int c1 = e.son0[c], c2 = e.son1[c];
          wg_copy(r1, r, Q, Eslot(e, side, c1));
          wg_copy(mr - r1, r, mv_at(Q, r1, 0), Eslot(e, side, c2));
        }
        if (c == root && e.parent[c] >= 0) {
          // E_{t0} <- R_{t0} [E_{t0}; 0]
          const int kpar = e.k[side][e.parent[c]];
          MV T = mv_col(L.W2, KM);
          wg_gemm(r, kpar, kc, 1.0, wslot(e.wR[side], c), Eslot(e, side, c), 0.0, T);
          count(e, fl_gemm(r, kpar, kc));
          wg_copy(r, kpar, T, Eslot(e, side, c));
        }
      }
    }
  }
  prof_stage(e, 4, tstage);
  // --- step 5: couplings of every admissible leaf touching the subtrees
  for (int side = 0; side < 2; ++side) {
    const int root = u.r0[side];
    const int *ptr = side == 0 ? e.rowptr : e.colptr;
    const int *idx = side == 0 ? e.rowidx : e.colidx;
    for (int lv = e.level[root]; lv < e.nlev; ++lv) {
      const int lo = dlo(e, root, lv), hi = dhi(e, root, lv);
      for (int c = lo; c < hi; ++c) {
        for (int p = ptr[c]; p < ptr[c + 1]; ++p) {
          const int b = idx[p];
          const int t = e.brow[b], s = e.bcol[b];
          if (side == 1 && in_sub(e, u.r0[0], t)) continue;
          const bool tin = in_sub(e, u.r0[0], t), sin = in_sub(e, u.r0[1], s);
          int Kt, Ks;
          MV St = mv_col(L.W2, KM);
          load_stilde(e, u, b, St, Kt, Ks);
          MV P = St;
          int rows = Kt;
          if (tin) {
            rows = e.wnewk[0][t];
            P = mv_col(L.W1, KM);
            wg_gemm(rows, Ks, Kt, 1.0, wslot(e.wR[0], t), St, 0.0, P);
            count(e, fl_gemm(rows, Ks, Kt));
          }
          MV Sd = Sslot(e, b);
          if (sin) {
            const int rs = e.wnewk[1][s];
            wg_gemm(rows, rs, Ks, 1.0, P, mv_t(wslot(e.wR[1], s)), 0.0, Sd);
            count(e, fl_gemm(rows, rs, Ks));
          } else {
            wg_copy(rows, Ks, P, Sd);
          }
        }
      }
    }
  }
  prof_stage(e, 5, tstage);
  // --- step 7: inadmissible leaves inside b0 receive X|_t Y|_s^*
  {
    const int root = u.r0[0];
    for (int lv = e.level[root]; lv < e.nlev; ++lv) {
      const int lo = dlo(e, root, lv), hi = dhi(e, root, lv);
      for (int c = lo; c < hi; ++c) {
        if (!is_leaf(e, c)) continue;
        for (int p = e.nrowptr[c]; p < e.nrowptr[c + 1]; ++p) {
          const int b = e.nrowidx[p];
          const int s = e.bcol[b];
          if (!in_sub(e, u.r0[1], s)) continue;
          wg_gemm(e.size[c], e.size[s], kp, 1.0, bufrows(e, u.buf[0], c),
                  mv_t(bufrows(e, u.buf[1], s)), 1.0, Nslot(e, b));
          count(e, fl_gemm(e.size[c], e.size[s], kp));
        }
      }
    }
  }
  prof_stage(e, 6, tstage);
  // --- step 6: commit ranks, R-factors of the new bases, refresh the path
  for (int side = 0; side < 2; ++side) {
    const int root = u.r0[side];
    for (int lv = e.level[root]; lv < e.nlev; ++lv) {
      const int lo = dlo(e, root, lv), hi = dhi(e, root, lv);
      for (int c = lo; c < hi; ++c) {
        const int r = e.wnewk[side][c];
        MV R = rhoslot(e, side, c);
        for (int q = threadIdx.x; q < r * r; q += blockDim.x) R(q % r, q / r) = (q % r == q / r) ? 1.0 : 0.0;
        if (threadIdx.x == 0) { e.k[side][c] = r; e.rho_m[side][c] = r; }
      }
    }
    __syncthreads();
    int c = e.parent[root];
    while (c >= 0) {
      const int kc = e.k[side][c];
      MV A = mv_col(L.W0, W0R);
      int m = 0;
      for (int sn = 0; sn < 2; ++sn) {
        const int ch = sn == 0 ? e.son0[c] : e.son1[c];
        const int mc = e.rho_m[side][ch];
        wg_gemm(mc, kc, e.k[side][ch], 1.0, rhoslot(e, side, ch), Eslot(e, side, ch), 0.0,
                mv_at(A, m, 0));
        m += mc;
      }
      wg_qr(m, kc, A, nullptr, L.red);
      count(e, fl_qr(m, kc) + fl_gemm(m, kc, e.k[side][e.son0[c]]));
      wg_extract_r(m, kc, A, rhoslot(e, side, c));
      if (threadIdx.x == 0) e.rho_m[side][c] = m < kc ? m : kc;
      __syncthreads();
      c = e.parent[c];
    }
  }
  prof_stage(e, 7, tstage);
}

// ====================================================== products with H^2
// Expanded basis of cluster t (through eq. (nested)) into buffer rows of t.
__device__ void task_expand(const DevEnv &e, int side, int t, int bo) {
  const int kt = e.k[side][t];
  MV out = bufrows(e, bo, t);
  if (is_leaf(e, t)) {
    wg_copy(e.size[t], kt, leafslot(e, side, t), out);
  } else {
    // T_c = E_c T_father (k_c x k_t) for the descendants, top-down, in xh
    for (int lv = e.level[t] + 1; lv < e.nlev; ++lv) {
      const int lo = dlo(e, t, lv), hi = dhi(e, t, lv);
      if (lo >= hi) break;
      const int tot = (hi - lo) * KC * kt;
      for (int q = threadIdx.x; q < tot; q += blockDim.x) {
        const int c = lo + q / (KC * kt);
        const int rem = q % (KC * kt);
        const int i = rem % KC, j = rem / KC;
        const int kc = e.k[side][c];
        if (i >= kc) continue;
        const int p = e.parent[c];
        MV Ec = Eslot(e, side, c);
        double s;
        if (p == t) s = Ec(i, j);
        else {
          MV Tp = xhslot(e.xh, p);
          s = 0.0;
          for (int l = 0; l < e.k[side][p]; ++l) s = fma(Ec(i, l), Tp(l, j), s);
        }
        xhslot(e.xh, c)(i, j) = s;
      }
      __syncthreads();
    }
    for (int lv = e.level[t] + 1; lv < e.nlev; ++lv) {
      const int lo = dlo(e, t, lv), hi = dhi(e, t, lv);
      if (lo >= hi) break;
      const int tot = (hi - lo) * LS * kt;
      for (int q = threadIdx.x; q < tot; q += blockDim.x) {
        const int c = lo + q / (LS * kt);
        if (!is_leaf(e, c)) continue;
        const int rem = q % (LS * kt);
        const int i = rem % LS, j = rem / LS;
        if (i >= e.size[c]) continue;
        MV V = leafslot(e, side, c);
        MV Tc = xhslot(e.xh, c);
        double s = 0.0;
        for (int l = 0; l < e.k[side][c]; ++l) s = fma(V(i, l), Tc(l, j), s);
        out(e.offset[c] - e.offset[t] + i, j) = s;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) e.bcols[bo] = kt;
  __syncthreads();
}

// out|_t = beta out|_t + alpha Z|_{t x s} in|_s (trans = 0) or
// out|_s = beta out|_s + alpha Z|_{t x s}^* in|_t (trans = 1) for the block
// b = (t, s): forward transformation, couplings, backward transformation,
// nearfield.
__device__ void task_bapply(const DevEnv &e, const Lds &L, int b, int trans, int bin, int bout,
                            double alpha, double beta) {
  double fl = 0.0;   // algorithmic flops of this thread
  const int m = e.bcols[bin];
  const int t = e.brow[b], s = e.bcol[b];
  const int sr = trans ? t : s, dr = trans ? s : t;
  const int ss = trans ? 0 : 1, ds = 1 - ss;
  MV out = bufrows(e, bout, dr);
  {
    const int rows = e.size[dr];
    for (int q = threadIdx.x; q < rows * m; q += blockDim.x) {
      const int i = q / m, j = q % m;
      out(i, j) = beta == 0.0 ? 0.0 : beta * out(i, j);
    }
  }
  __syncthreads();
  // forward transformation over the source subtree
  for (int lv = e.nlev - 1; lv >= e.level[sr]; --lv) {
    const int lo = dlo(e, sr, lv), hi = dhi(e, sr, lv);
    if (lo >= hi) continue;
    const int tot = (hi - lo) * KC * m;
    for (int q = threadIdx.x; q < tot; q += blockDim.x) {
      const int c = lo + q / (KC * m);
      const int rem = q % (KC * m);
      const int i = rem / m, j = rem % m;
      const int kc = e.k[ss][c];
      if (i >= kc) continue;
      double acc = 0.0;
      if (is_leaf(e, c)) {
        MV V = leafslot(e, ss, c);
        MV x = bufrows(e, bin, c);
        for (int l = 0; l < e.size[c]; ++l) acc = fma(V(l, i), x(l, j), acc);
        fl += 2.0 * e.size[c];
      } else {
        for (int sn = 0; sn < 2; ++sn) {
          const int ch = sn == 0 ? e.son0[c] : e.son1[c];
          MV Ec = Eslot(e, ss, ch);
          MV xc = xhslot(e.xh, ch);
          for (int l = 0; l < e.k[ss][ch]; ++l) acc = fma(Ec(l, i), xc(l, j), acc);
          fl += 2.0 * e.k[ss][ch];
        }
      }
      xhslot(e.xh, c)(i, j) = acc;
    }
    __syncthreads();
  }
  // couplings into the destination subtree
  const int *ptr = trans ? e.colptr : e.rowptr;
  const int *idx = trans ? e.colidx : e.rowidx;
  for (int lv = e.level[dr]; lv < e.nlev; ++lv) {
    const int lo = dlo(e, dr, lv), hi = dhi(e, dr, lv);
    if (lo >= hi) break;
    const int tot = (hi - lo) * KC * m;
    for (int q = threadIdx.x; q < tot; q += blockDim.x) {
      const int c = lo + q / (KC * m);
      const int rem = q % (KC * m);
      const int i = rem / m, j = rem % m;
      if (i >= e.k[ds][c]) continue;
      double acc = 0.0;
      for (int p = ptr[c]; p < ptr[c + 1]; ++p) {
        const int bb = idx[p];
        const int o = trans ? e.brow[bb] : e.bcol[bb];
        if (!in_sub(e, sr, o)) continue;
        MV S = Sslot(e, bb);
        MV xo = xhslot(e.xh, o);
        const int ko = e.k[ss][o];
        if (!trans) { for (int l = 0; l < ko; ++l) acc = fma(S(i, l), xo(l, j), acc); }
        else { for (int l = 0; l < ko; ++l) acc = fma(S(l, i), xo(l, j), acc); }
        fl += 2.0 * ko;
      }
      xhslot(e.yh, c)(i, j) = acc;
    }
    __syncthreads();
  }
  // backward transformation
  for (int lv = e.level[dr] + 1; lv < e.nlev; ++lv) {
    const int lo = dlo(e, dr, lv), hi = dhi(e, dr, lv);
    if (lo >= hi) break;
    const int tot = (hi - lo) * KC * m;
    for (int q = threadIdx.x; q < tot; q += blockDim.x) {
      const int c = lo + q / (KC * m);
      const int rem = q % (KC * m);
      const int i = rem / m, j = rem % m;
      if (i >= e.k[ds][c]) continue;
      const int p = e.parent[c];
      MV Ec = Eslot(e, ds, c);
      MV yp = xhslot(e.yh, p);
      double acc = xhslot(e.yh, c)(i, j);
      for (int l = 0; l < e.k[ds][p]; ++l) acc = fma(Ec(i, l), yp(l, j), acc);
      fl += 2.0 * e.k[ds][p];
      xhslot(e.yh, c)(i, j) = acc;
    }
    __syncthreads();
  }
  // leaves: basis part and nearfield
  const int *nptr = trans ? e.ncolptr : e.nrowptr;
  const int *nidx = trans ? e.ncolidx : e.nrowidx;
  for (int lv = e.level[dr]; lv < e.nlev; ++lv) {
    const int lo = dlo(e, dr, lv), hi = dhi(e, dr, lv);
    if (lo >= hi) break;
    const int tot = (hi - lo) * LS * m;
    for (int q = threadIdx.x; q < tot; q += blockDim.x) {
      const int c = lo + q / (LS * m);
      if (!is_leaf(e, c)) continue;
      const int rem = q % (LS * m);
      const int i = rem / m, j = rem % m;
      if (i >= e.size[c]) continue;
      double acc = 0.0;
      MV V = leafslot(e, ds, c);
      MV yc = xhslot(e.yh, c);
      for (int l = 0; l < e.k[ds][c]; ++l) acc = fma(V(i, l), yc(l, j), acc);
      fl += 2.0 * e.k[ds][c];
      for (int p = nptr[c]; p < nptr[c + 1]; ++p) {
        const int bb = nidx[p];
        const int o = trans ? e.brow[bb] : e.bcol[bb];
        if (!in_sub(e, sr, o)) continue;
        MV N = Nslot(e, bb);
        MV xo = bufrows(e, bin, o);
        const int no = e.size[o];
        if (!trans) { for (int l = 0; l < no; ++l) acc = fma(N(i, l), xo(l, j), acc); }
        else { for (int l = 0; l < no; ++l) acc = fma(N(l, i), xo(l, j), acc); }
        fl += 2.0 * no;
      }
      MV oc = bufrows(e, bout, c);
      oc(i, j) = oc(i, j) + alpha * acc;
    }
  }
  __syncthreads();
  fl = wg_sum(fl, L.red);
  count(e, fl);
  if (threadIdx.x == 0) e.bcols[bout] = m;
  __syncthreads();
}

// out|_cl = alpha in|_cl op(S_b)
__device__ void task_rmul_s(const DevEnv &e, int bin, int bout, int b, int transS, int cl, double alpha) {
  const int kt = e.k[0][e.brow[b]], ks = e.k[1][e.bcol[b]];
  const int kin = transS ? ks : kt, kout = transS ? kt : ks;
  MV S = Sslot(e, b);
  MV Sop = transS ? mv_t(S) : S;
  wg_gemm(e.size[cl], kout, kin, alpha, bufrows(e, bin, cl), Sop, 0.0, bufrows(e, bout, cl));
  count(e, fl_gemm(e.size[cl], kout, kin));
  if (threadIdx.x == 0) e.bcols[bout] = kout;
  __syncthreads();
}

__device__ void task_copy_near(const DevEnv &e, int b, int bout, double alpha) {
  const int t = e.brow[b], s = e.bcol[b];
  MV N = Nslot(e, b);
  MV out = bufrows(e, bout, t);
  const int mt = e.size[t], ns = e.size[s];
  for (int q = threadIdx.x; q < mt * ns; q += blockDim.x) {
    const int i = q % mt, j = q / mt;
    out(i, j) = alpha * N(i, j);
  }
  if (threadIdx.x == 0) e.bcols[bout] = ns;
  __syncthreads();
}

__device__ void task_ident(const DevEnv &e, int cl, int bo, int c0, int nc) {
  MV out = bufrows(e, bo, cl);
  const int m = e.size[cl];
  for (int q = threadIdx.x; q < m * nc; q += blockDim.x) {
    const int i = q / nc, j = q % nc;
    out(i, j) = (i == c0 + j) ? 1.0 : 0.0;
  }
  if (threadIdx.x == 0) e.bcols[bo] = nc;
  __syncthreads();
}

__device__ void task_near_add(const DevEnv &e, int b, int bu, int bv, double alpha) {
  const int t = e.brow[b], s = e.bcol[b];
  wg_gemm(e.size[t], e.size[s], e.bcols[bu], alpha, bufrows(e, bu, t), mv_t(bufrows(e, bv, s)), 1.0,
          Nslot(e, b));
  count(e, fl_gemm(e.size[t], e.size[s], e.bcols[bu]));
}

__device__ void task_temp_init(const DevEnv &e, int bu, int bv, int t, int r) {
  MV U = bufrows(e, bu, t), V = bufrows(e, bv, r);
  const int mt = e.size[t], mr = e.size[r];
  for (int q = threadIdx.x; q < mt * BC; q += blockDim.x) U(q / BC, q % BC) = 0.0;
  for (int q = threadIdx.x; q < mr * BC; q += blockDim.x) V(q / BC, q % BC) = 0.0;
  if (threadIdx.x == 0) { e.bcols[bu] = 0; e.bcols[bv] = 0; }
  __syncthreads();
}

// Truncated addition of the zero-extended emission (U on rows t', V on rows
// r') to the temporary low-rank matrix (tU, tV) on (tT, rT).
__device__ void task_temp_add(const DevEnv &e, const Lds &L, const Task &tk) {
  const int tu = tk.i[0], tv = tk.i[1], tp = tk.i[2], rp = tk.i[3], bu = tk.i[4], bv = tk.i[5];
  const int tT = tk.i[6], rT = tk.i[7];
  const int k1 = e.bcols[tu], k2 = e.bcols[bu];
  const int kk = k1 + k2;
  if (kk == 0) return;
  const int mt = e.size[tT], mr = e.size[rT];
  MV A = bufrows(e, B_A, tT), B = bufrows(e, B_B, rT);
  {
    MV TU = bufrows(e, tu, tT), TV = bufrows(e, tv, rT);
    const int at = e.offset[tp] - e.offset[tT], ar = e.offset[rp] - e.offset[rT];
    const int nt = e.size[tp], nr = e.size[rp];
    MV U = bufrows(e, bu, tp), V = bufrows(e, bv, rp);
    for (int q = threadIdx.x; q < mt * kk; q += blockDim.x) {
      const int i = q / kk, j = q % kk;
      A(i, j) = j < k1 ? TU(i, j) : ((i >= at && i < at + nt) ? U(i - at, j - k1) : 0.0);
    }
    for (int q = threadIdx.x; q < mr * kk; q += blockDim.x) {
      const int i = q / kk, j = q % kk;
      B(i, j) = j < k1 ? TV(i, j) : ((i >= ar && i < ar + nr) ? V(i - ar, j - k1) : 0.0);
    }
    __syncthreads();
  }
  double *ta = L.tau, *tb = L.tau + KM;
  wg_qr(mt, kk, A, ta, L.red);
  wg_qr(mr, kk, B, tb, L.red);
  const int qa = mt < kk ? mt : kk, qb = mr < kk ? mr : kk;
  MV C = mv_col(L.W1, KM), J = mv_col(L.W2, KM);
  {
    // C = Ra Rb^T (qa x qb), J = I
    for (int q = threadIdx.x; q < qa * qb; q += blockDim.x) {
      const int i = q % qa, j = q / qa;
      double s = 0.0;
      for (int l = (i > j ? i : j); l < kk; ++l) s = fma(A(i, l), B(j, l), s);
      C(i, j) = s;
    }
    for (int q = threadIdx.x; q < qb * qb; q += blockDim.x) J(q % qb, q / qb) = (q % qb == q / qb) ? 1.0 : 0.0;
    __syncthreads();
  }
  wg_jacobi(qa, qb, C, &J, L.iw);
  {
    const double bmin = qa < qb ? qa : qb;   // both singular vector sets: + 14 b^3
    count(e, fl_qr(mt, kk) + fl_qr(mr, kk) + fl_gemm(qa, qb, kk) + fl_svd(qa, qb) + 14.0 * bmin * bmin * bmin);
  }
  int *ord = L.iw + KM;
  wg_colnorms_sorted(qa, qb, C, L.sig, ord);
  double tau = 0.0;
  if (e.mode == 0) {
    double s2 = 0.0;
    for (int j = 0; j < qb; ++j) s2 += L.sig[j] * L.sig[j];
    tau = e.eps * sqrt(s2);
  } else if (e.mode == 1) {
    tau = e.eps * (qb > 0 ? L.sig[ord[0]] : 0.0);
  }
  int r = 0;
  for (int j = 0; j < qb; ++j) r += L.sig[ord[j]] > tau ? 1 : 0;
  if (r > e.rank_cap) { set_error(e, E_RANK_CAP, tT); return; }
  MV Qa = bufrows(e, B_W, tT), Qb = bufrows(e, B_WP, rT);
  wg_form_q(mt, kk, A, ta, Qa);
  wg_form_q(mr, kk, B, tb, Qb);
  MV TU = bufrows(e, tu, tT), TV = bufrows(e, tv, rT);
  for (int q = threadIdx.x; q < mt * r; q += blockDim.x) {
    const int i = q / r, j = q % r;
    const int c = ord[j];
    double s = 0.0;
    for (int l = 0; l < qa; ++l) s = fma(Qa(i, l), C(l, c), s);
    TU(i, j) = s;
  }
  for (int q = threadIdx.x; q < mr * r; q += blockDim.x) {
    const int i = q / r, j = q % r;
    const int c = ord[j];
    double s = 0.0;
    for (int l = 0; l < qb; ++l) s = fma(Qb(i, l), J(l, c), s);
    TV(i, j) = s;
  }
  count(e, fl_qr(mt, kk) + fl_qr(mr, kk) + fl_gemm(mt, r, qa) + fl_gemm(mr, r, qb));
  if (threadIdx.x == 0) { e.bcols[tu] = r; e.bcols[tv] = r; }
  __syncthreads();
}

__device__ void task_potrf(const DevEnv &e, const Lds &L, int bcc, int t) {
  const int info = wg_potrf(e.size[t], Nslot(e, bcc), L.iw);
  count(e, (double)e.size[t] * e.size[t] * e.size[t] / 3.0);
  if (info) set_error(e, E_NOT_SPD, t);
}

__device__ void task_trsm(const DevEnv &e, int b, int bcc) {
  const int r = e.brow[b], c = e.brow[bcc];
  wg_trsm_right_lt(e.size[r], e.size[c], Nslot(e, bcc), Nslot(e, b));
  count(e, (double)e.size[r] * e.size[c] * e.size[c]);
}

__device__ void task_trsv(const DevEnv &e, int bcc, int bi, int trans) {
  const int c = e.brow[bcc];
  wg_trsv_lower(e.size[c], e.bcols[bi], Nslot(e, bcc), bufrows(e, bi, c), trans);
  count(e, (double)e.size[c] * e.size[c] * e.bcols[bi]);
}

__device__ void task_sub(const DevEnv &e, int ba, int bb, int bo, int cl) {
  const int m = e.bcols[ba];
  MV A = bufrows(e, ba, cl), B = bufrows(e, bb, cl), O = bufrows(e, bo, cl);
  const int rows = e.size[cl];
  for (int q = threadIdx.x; q < rows * m; q += blockDim.x) O(q / m, q % m) = A(q / m, q % m) - B(q / m, q % m);
  if (threadIdx.x == 0) e.bcols[bo] = m;
  __syncthreads();
}

__device__ void task_copy(const DevEnv &e, int ba, int bo, int cl) {
  const int m = e.bcols[ba];
  MV A = bufrows(e, ba, cl), O = bufrows(e, bo, cl);
  const int rows = e.size[cl];
  for (int q = threadIdx.x; q < rows * m; q += blockDim.x) O(q / m, q % m) = A(q / m, q % m);
  if (threadIdx.x == 0) e.bcols[bo] = m;
  __syncthreads();
}

// ============================================================ interpreter
__global__ __launch_bounds__(NT) void k_interp(const Task *__restrict__ tasks, int ntask,
                                               const DevEnv *__restrict__ env) {
  extern __shared__ double lds_raw[];
  const DevEnv &e = *env;
  const Lds L = lds_layout(lds_raw);
  for (int it = 0; it < ntask; ++it) {
    __syncthreads();
    if (e.err[0] != 0) return;
    const Task tk = tasks[it];
    const unsigned long long t0 = e.prof ? wall_clock64() : 0ull;
    switch (tk.op) {
      case OP_ADDLR: task_addlr(e, L, tk.i[0], tk.i[1], tk.i[2]); break;
      case OP_EXPAND: task_expand(e, tk.i[0], tk.i[1], tk.i[2]); break;
      case OP_BAPPLY: task_bapply(e, L, tk.i[0], tk.i[1], tk.i[2], tk.i[3], tk.alpha, tk.beta); break;
      case OP_RMUL_S: task_rmul_s(e, tk.i[0], tk.i[1], tk.i[2], tk.i[3], tk.i[4], tk.alpha); break;
      case OP_COPY_NEAR: task_copy_near(e, tk.i[0], tk.i[1], tk.alpha); break;
      case OP_IDENT: task_ident(e, tk.i[0], tk.i[1], tk.i[2], tk.i[3]); break;
      case OP_NEAR_ADD: task_near_add(e, tk.i[0], tk.i[1], tk.i[2], tk.alpha); break;
      case OP_TEMP_INIT: task_temp_init(e, tk.i[0], tk.i[1], tk.i[2], tk.i[3]); break;
      case OP_TEMP_ADD: task_temp_add(e, L, tk); break;
      case OP_POTRF: task_potrf(e, L, tk.i[0], tk.i[1]); break;
      case OP_TRSM: task_trsm(e, tk.i[0], tk.i[1]); break;
      case OP_TRSV: task_trsv(e, tk.i[0], tk.i[1], tk.i[2]); break;
      case OP_SUB: task_sub(e, tk.i[0], tk.i[1], tk.i[2], tk.i[3]); break;
      case OP_COPY: task_copy(e, tk.i[0], tk.i[1], tk.i[2]); break;
      default: set_error(e, E_ARG, tk.op); break;
    }
    if (e.prof && threadIdx.x == 0 && tk.op > 0 && tk.op < 32) {
      e.prof[PROF_COUNT + tk.op] += 1;
      e.prof[PROF_TICKS + tk.op] += wall_clock64() - t0;
    }
  }
}

// ======================================================== helper kernels
// dst buffer rows (cluster order, row-major BC) <- src (original order,
// column-major n x ncol, leading dimension ld), rows [r0, r0+nr) of the buffer.
__global__ void k_gather(int nr, int r0, int ncol, const int64_t *__restrict__ perm,
                         const double *__restrict__ src, long ld, double *__restrict__ dst,
                         int *bcols, int bi) {
  const long tot = (long)nr * ncol;
  for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < tot; q += (long)gridDim.x * blockDim.x) {
    const int i = (int)(q % nr), j = (int)(q / nr);
    const long row = r0 + i;
    dst[row * BC + j] = src[(perm ? perm[row] : i) + j * ld];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) bcols[bi] = ncol;
}

// y (original order) = alpha * buf + beta * y
__global__ void k_scatter(int n, int ncol, const int64_t *__restrict__ perm, const double *__restrict__ src,
                          double *__restrict__ y, long ld, double alpha, double beta) {
  const long tot = (long)n * ncol;
  for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < tot; q += (long)gridDim.x * blockDim.x) {
    const int i = (int)(q % n), j = (int)(q / n);
    double *p = y + perm[i] + j * ld;
    const double v = alpha * src[(long)i * BC + j];
    *p = beta == 0.0 ? v : fma(beta, *p, v);
  }
}

__global__ void k_fill_int(int *p, int n, int v) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) p[q] = v;
}

// CSR product y = A x (one thread per row).
__global__ void k_spmv(int n, const int64_t *__restrict__ rp, const int *__restrict__ ci,
                       const double *__restrict__ v, const double *__restrict__ x, double *__restrict__ y) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s = fma(v[p], x[ci[p]], s);
    y[i] = s;
  }
}

// Deterministic dot product: per-block partial sums, then one block.
__global__ void k_dot_partial(int n, const double *__restrict__ a, const double *__restrict__ b,
                              double *__restrict__ part) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) s = fma(a[i], b[i], s);
  s = wave_sum(s);
  if (lane_id() == 0) red[wave_id()] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < num_waves(); ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

__global__ void k_dot_final(int np, const double *__restrict__ part, double *__restrict__ out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
  s = wave_sum(s);
  if (lane_id() == 0) red[wave_id()] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < num_waves(); ++w) t += red[w];
    *out = t;
  }
}

// PCG vector updates with scalars kept on the device.
// sc[0] = r.z, sc[1] = p.q, sc[2] = r.z (new), sc[3] = r.r
__global__ void k_pcg_update_xr(int n, const double *__restrict__ sc, const double *__restrict__ p,
                                const double *__restrict__ q, double *__restrict__ x, double *__restrict__ r) {
  const double alpha = sc[0] / sc[1];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    x[i] = fma(alpha, p[i], x[i]);
    r[i] = fma(-alpha, q[i], r[i]);
  }
}

__global__ void k_pcg_update_p(int n, double *__restrict__ sc, const double *__restrict__ z,
                               double *__restrict__ p) {
  const double beta = sc[2] / sc[0];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = fma(beta, p[i], z[i]);
}

__global__ void k_copy_scalar(double *dst, const double *src) { *dst = *src; }

}  // namespace h2
