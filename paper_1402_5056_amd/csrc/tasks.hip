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

// Nearest bfloat16 value (ties to even) of v, returned as a double.
__device__ __forceinline__ double round_bf16(double v) {
  unsigned int u = __float_as_uint((float)v);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (double)__uint_as_float(u & 0xffff0000u);
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
// The update runs level by level.  Inside one level the clusters of both
// subtrees (for the weights also the predecessors of t0 and s0) depend on
// each other only through the previous level, so they are processed
// concurrently, one wave per cluster, with a workgroup barrier per level.

constexpr int NWAVE = NT / 64;
constexpr int WREG = 2304;      // doubles of LDS per wave for work matrices
constexpr int WSMALL = 256;     // doubles of LDS per wave for vectors
constexpr int WGLOB = 65536;    // doubles of global scratch per wave (overflow)
constexpr int TEMP_WAVE_MAX = 16384;   // larger truncated additions run on the whole workgroup
constexpr int PRECOND_MIN = 6;  // SVDs with more columns are QR-preconditioned
constexpr size_t LDS_WAVE_DOUBLES = (size_t)NWAVE * (WREG + WSMALL);
constexpr size_t LDS_TOTAL_DOUBLES = LDS_WAVE_DOUBLES > LDS_DOUBLES ? LDS_WAVE_DOUBLES : LDS_DOUBLES;

struct Upd {
  int r0[2];   // t0, s0
  int buf[2];  // X, Y buffers
  int kp;
};

struct Wv {
  double *reg;   // LDS work area
  double *sig;   // LDS, 64 doubles
  int *ord;      // LDS, 128 ints
  double *glob;  // global overflow area
  int w;
};

__device__ __forceinline__ Wv wave_areas_of(double *lds, const DevEnv &e, int w) {
  Wv W;
  W.w = w;
  W.reg = lds + W.w * (WREG + WSMALL);
  W.sig = W.reg + WREG;
  W.ord = reinterpret_cast<int *>(W.sig + 64);
  W.glob = e.wscr + (long)W.w * WGLOB;
  return W;
}
__device__ __forceinline__ Wv wave_areas(double *lds, const DevEnv &e) {
  Wv W;
  W.w = wave_id();
  W.reg = lds + W.w * (WREG + WSMALL);
  W.sig = W.reg + WREG;
  W.ord = reinterpret_cast<int *>(W.sig + 64);
  W.glob = e.wscr + (long)W.w * WGLOB;
  return W;
}

// Bump allocation of a wave's work matrices: LDS while it fits, then the
// wave's global overflow area.  Odd leading dimensions spread LDS banks.
// A request beyond the overflow area reports E_SCRATCH and reuses the start
// of the area, so that every access stays in bounds.
struct WvAlloc {
  double *lds, *glob;
  int *err;
  int lused, gused;
  int lcap = WREG;   // doubles of LDS available at lds
  __device__ MV take(int m, int n) {
    const int ld = m | 1;
    const int need = ld * (n > 0 ? n : 1);
    double *p;
    if (lused + need <= lcap) { p = lds + lused; lused += need; }
    else if (gused + need <= WGLOB) { p = glob + gused; gused += need; }
    else {
      if (lane_id() == 0) { err[1] = need; err[0] = E_SCRATCH; }
      p = glob;
    }
    return mv_col(p, ld);
  }
};
__device__ __forceinline__ WvAlloc wv_alloc(const DevEnv &e, const Wv &W) {
  return WvAlloc{W.reg, W.glob, e.err, 0, 0};
}

// Algorithmic flops of a wave's work in update step st (and, when profiling,
// per step); bytes: algorithmic bytes of the H^2 data the step reads and
// writes (profiling only).
__device__ __forceinline__ void bytes_w(const DevEnv &e, int st, double b) {
  if (e.prof && lane_id() == 0) atomicAdd(&e.prof[PROF_SBYTES + st], (unsigned long long)b);
}
__device__ __forceinline__ void count_w(const DevEnv &e, const Wv &W, int st, double f) {
  if (e.prof && lane_id() == 0) atomicAdd(&e.prof[PROF_SFLOPS + st], (unsigned long long)f);
  if (lane_id() == 0 && e.flops) e.flops[1 + W.w] += f;
}

// Per-wave tracing: ticks spent in a sub-step (summed over waves) and event
// counts.  No-ops unless profiling is enabled.
enum : int {
  WT_RF_BUILD = 0, WT_RF_QR, WT_W_OMEGA, WT_W_STACK, WT_W_QR, WT_RC_BUILD, WT_RC_M, WT_RC_SVD,
  WT_RC_OUT, WT_CPL, WT_REFRESH, WT_NEAR,
  WC_W_CALLS = 16, WC_W_BLOCKS, WC_W_NONEMPTY, WC_QR_CALLS, WC_QR_COLS, WC_QR_ROWS, WC_REFRESH
};
__device__ __forceinline__ unsigned long long wt_now(const DevEnv &e) {
  return e.prof ? wall_clock64() : 0ull;
}
__device__ __forceinline__ void wt_add(const DevEnv &e, int slot, unsigned long long &t) {
  if (e.prof) {
    const unsigned long long now = wall_clock64();
    if (lane_id() == 0) atomicAdd(&e.prof[PROF_WAVE + slot], now - t);
    t = now;
  }
}
__device__ __forceinline__ void wc_add(const DevEnv &e, int slot, long v) {
  if (e.prof && lane_id() == 0) atomicAdd(&e.prof[PROF_WAVE + slot], (unsigned long long)v);
}
__device__ __forceinline__ void wv_qr_traced(const DevEnv &e, int m, int n, MV A) {
  wc_add(e, WC_QR_CALLS, 1);
  wc_add(e, WC_QR_COLS, m < n ? m : n);
  wc_add(e, WC_QR_ROWS, m);
  wv_qr(m, n, A, nullptr);
}

// R-factor of the (possibly extended) basis of cluster c.
__device__ __forceinline__ MV rho_of(const DevEnv &e, const Upd &u, int side, int c, int &m) {
  if (in_sub(e, u.r0[side], c)) { m = e.wrho_m[side][c]; return wslot(e.wrho[side], c); }
  m = e.rho_m[side][c];
  return rhoslot(e, side, c);
}

// Entry (i, j) of the extended coupling S~_b (Section 5, three rules).
struct SExt {
  MV S;
  int kt, ks, Kt, Ks;
  bool tin, sin;
  __device__ __forceinline__ double operator()(int i, int j) const {
    if (i < kt && j < ks) return S(i, j);
    return (tin && sin && i >= kt && j >= ks && (i - kt) == (j - ks)) ? 1.0 : 0.0;
  }
};
__device__ __forceinline__ SExt sext(const DevEnv &e, const Upd &u, int b) {
  SExt x;
  const int t = e.brow[b], s = e.bcol[b];
  x.S = Sslot(e, b);
  x.kt = e.k[0][t]; x.ks = e.k[1][s];
  x.tin = in_sub(e, u.r0[0], t); x.sin = in_sub(e, u.r0[1], s);
  x.Kt = x.kt + (x.tin ? u.kp : 0);
  x.Ks = x.ks + (x.sin ? u.kp : 0);
  return x;
}

// Step 1: R-factor of the extended basis of cluster c (one wave).
__device__ void wv_rfactor(const DevEnv &e, const Upd &u, const Wv &W, int side, int c) {
  const int lane = lane_id();
  unsigned long long tw = wt_now(e);
  const int kc = e.k[side][c], K = kc + u.kp;
  WvAlloc al = wv_alloc(e, W);
  int m;
  MV A;
  double fl = 0.0;
  if (is_leaf(e, c)) {
    m = e.size[c];
    A = al.take(m, K);
    MV V = leafslot(e, side, c), F = bufrows(e, u.buf[side], c);
    for (int q = lane; q < m * K; q += 64) {
      const int i = q % m, j = q / m;
      A(i, j) = j < kc ? V(i, j) : F(i, j - kc);
    }
  } else {
    const int c1 = e.son0[c], c2 = e.son1[c];
    const int m1 = e.wrho_m[side][c1], m2 = e.wrho_m[side][c2];
    m = m1 + m2;
    A = al.take(m, K);
    for (int sn = 0; sn < 2; ++sn) {
      const int ch = sn == 0 ? c1 : c2, mc = sn == 0 ? m1 : m2, off = sn == 0 ? 0 : m1;
      const int kch = e.k[side][ch];
      MV Rc = wslot(e.wrho[side], ch), Ec = Eslot(e, side, ch);
      for (int q = lane; q < mc * K; q += 64) {
        const int i = q % mc, j = q / mc;
        double sacc = 0.0;
        if (j < kc) { sacc = dotc(0, kch, [&](int l) { return Rc(i, l); }, [&](int l) { return Ec(l, j); }, sacc); }
        else sacc = Rc(i, kch + (j - kc));
        A(off + i, j) = sacc;
      }
      fl += fl_gemm(mc, kc, kch);
    }
  }
  wave_sync();
  wt_add(e, WT_RF_BUILD, tw);
  wv_qr_traced(e, m, K, A);
  wt_add(e, WT_RF_QR, tw);
  const int mr = m < K ? m : K;
  MV R = wslot(e.wrho[side], c);
  for (int q = lane; q < mr * K; q += 64) {
    const int i = q % mr, j = q / mr;
    R(i, j) = j >= i ? A(i, j) : 0.0;
  }
  if (lane == 0) e.wrho_m[side][c] = mr;
  count_w(e, W, ST_A4, fl + fl_qr(m, K));
  // leaf: V_t and the update rows X|t (Y|s) read once
  if (is_leaf(e, c)) bytes_w(e, ST_A4, 8.0 * e.size[c] * K);
  wave_sync();
}

// Steps 2/3: weight matrix B~_t (Section 4; all blocks of row(t), Section 5),
// built by a stack of scaled blocks compressed with QR (one wave).  For a
// block b the stacked rows are G_b = rho_o S~_b^* (row side, rho_o the column
// R-factor of s) or rho_o S~_b (column side, rho_o the row R-factor of t);
// the block-relative scale is 1 / ||rho_t S~_b rho_s^*||_F = 1 / ||G_b rho^*||_F
// with rho the R-factor of the cluster itself.  The last rows are
// B~_parent diag(E_t, I)^*.  Since only the Gram matrix of the stack matters
// (the R-factor is determined up to a left orthogonal factor, which changes
// neither the left singular vectors of V^_t B~_t^* nor the stacks of the
// sons), the work can be split:
//   W_FULL   block rows and parent rows;
//   W_ROWS   block rows only (R-factor stored in the weight slot of t);
//   W_CHAIN  the stored R-factor of the block rows and the parent rows.
// The metadata of all blocks of the row is read lane-parallel; blocks whose
// extended coupling is identically zero add nothing and are skipped; the
// operands of a used block are staged in LDS before its rows are formed.
enum : int { W_FULL = 0, W_ROWS = 1, W_CHAIN = 2 };

__device__ __forceinline__ int rd_lane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ void wv_weight(const DevEnv &e, const Upd &u, const Wv &W, int side, int t, bool insub,
                          int wmode) {
  const int lane = lane_id();
  unsigned long long tw = wt_now(e);
  wc_add(e, WC_W_CALLS, 1);
  const int kt = e.k[side][t];
  const int Kt = kt + (insub ? u.kp : 0);
  const int cap = Kt + KM;          // any single block fits after a compression
  WvAlloc al = wv_alloc(e, W);
  MV A = al.take(cap, Kt);
  int m = 0, mrows = 0;
  double fl = 0.0;
  MV Wt = wslot(e.wB[side], t);
  if (wmode == W_CHAIN) {
    m = e.wB_m[side][t];
    for (int q = lane; q < m * Kt; q += 64) A(q % m, q / m) = Wt(q % m, q / m);
    wave_sync();
  } else {
    int mown = 0;
    MV Rown{nullptr, 0, 0};
    if (e.mode == 0) {
      MV Rg = rho_of(e, u, side, t, mown);
      Rown = al.take(mown, Kt);
      for (int q = lane; q < mown * Kt; q += 64) Rown(q % mown, q / mown) = Rg(q % mown, q / mown);
    }
    const WvAlloc blk0 = al;        // per-block staging starts here
    const int *ptr = side == 0 ? e.rowptr : e.colptr;
    const int *idx = side == 0 ? e.rowidx : e.colidx;
    const int p0 = ptr[t], nb = ptr[t + 1] - p0;
    for (int base = 0; base < nb; base += 64) {
      // lane-parallel metadata of up to 64 blocks
      int b = 0, mo = 0, kbt = 0, kbs = 0, fx = 0;
      bool use = false;
      if (base + lane < nb) {
        b = idx[p0 + base + lane];
        const int bt = e.brow[b], bs = e.bcol[b];
        kbt = e.k[0][bt];
        kbs = e.k[1][bs];
        const bool tin = in_sub(e, u.r0[0], bt), sin = in_sub(e, u.r0[1], bs);
        const bool ext = tin && sin && u.kp > 0;
        fx = (tin ? 1 : 0) | (sin ? 2 : 0) | (ext ? 4 : 0);
        use = ((kbt > 0 && kbs > 0) || ext) && !(e.mode == 0 && mown == 0);
        if (use) {
          const int other = side == 0 ? bs : bt;
          mo = in_sub(e, u.r0[1 - side], other) ? e.wrho_m[1 - side][other] : e.rho_m[1 - side][other];
          use = mo > 0;
        }
      }
      wc_add(e, WC_W_BLOCKS, nb - base < 64 ? nb - base : 64);
      unsigned long long mask = __ballot(use);
      while (mask != 0ull) {
        const int l = __ffsll((long long)mask) - 1;
        mask &= mask - 1ull;
        const int bb = rd_lane(b, l), mob = rd_lane(mo, l), kt_b = rd_lane(kbt, l), ks_b = rd_lane(kbs, l);
        const int f = rd_lane(fx, l);
        const bool tin = f & 1, sin = f & 2, ext = f & 4;
        const int other = side == 0 ? e.bcol[bb] : e.brow[bb];
        int mo2;
        MV Rog = rho_of(e, u, 1 - side, other, mo2);
        const int Kbt = kt_b + (tin ? u.kp : 0), Kbs = ks_b + (sin ? u.kp : 0);
        const int Ko = side == 0 ? Kbs : Kbt;
        // stage T = S~_b (row side) or S~_b^* (column side), Kt x Ko, and rho_o
        WvAlloc sa = blk0;
        MV T = sa.take(Kt, Ko), Ro = sa.take(mob, Ko);
        const MV S = Sslot(e, bb);
        for (int q = lane; q < Kt * Ko; q += 64) {
          const int j = q % Kt, c = q / Kt;
          const int i0 = side == 0 ? j : c, j0 = side == 0 ? c : j;   // entry (i0, j0) of S~_b
          double v;
          if (i0 < kt_b && j0 < ks_b) v = S(i0, j0);
          else v = (ext && i0 >= kt_b && j0 >= ks_b && i0 - kt_b == j0 - ks_b) ? 1.0 : 0.0;
          T(j, c) = v;
        }
        for (int q = lane; q < mob * Ko; q += 64) Ro(q % mob, q / mob) = Rog(q % mob, q / mob);
        if (m + mob > cap) {
          wt_add(e, WT_W_STACK, tw);
          wv_qr_traced(e, m, Kt, A);    // ends with wave_sync (also for the staging)
          const int mc = m < Kt ? m : Kt;
          for (int q = lane; q < mc * mc; q += 64) { const int i = q % mc, j = q / mc; if (i > j) A(i, j) = 0.0; }
          m = mc;
          wt_add(e, WT_W_QR, tw);
        }
        wave_sync();
        wc_add(e, WC_W_NONEMPTY, 1);
        // the coupling of a block above the subtrees is read once for the
        // path weights (those touching the subtrees count in step a7)
        if (!insub) bytes_w(e, ST_A5, 8.0 * kt_b * ks_b);
        // G_b = rho_o T^* into rows m .. m+mo of the stack
        wv_mm_f64(mob, Kt, Ko, [&](int i, int c) { return Ro(i, c); }, [&](int c, int j) { return T(j, c); },
                  [&](int i, int j, double v) { A(m + i, j) = v; });
        wave_sync();
        fl += fl_gemm(mob, Kt, Ko);
        if (e.mode == 0) {
          double f2 = 0.0;
          wv_mm_f64(mob, mown, Kt, [&](int i, int j) { return A(m + i, j); }, [&](int j, int a) { return Rown(a, j); },
                    [&](int, int, double v) { f2 = fma(v, v, f2); });
          f2 = wave_sum64(f2);
          fl += fl_gemm(mob, mown, Kt);
          if (f2 == 0.0) { wt_add(e, WT_W_OMEGA, tw); continue; }
          const double wsc = 1.0 / sqrt(f2);
          for (int q = lane; q < mob * Kt; q += 64) A(m + q % mob, q / mob) *= wsc;
          wave_sync();
        }
        wt_add(e, WT_W_OMEGA, tw);
        m += mob;
        mrows += mob;
      }
    }
  }
  const int par = e.parent[t];
  if (wmode != W_ROWS && par >= 0) {
    const int kpar = e.k[side][par];
    const int mp = e.wB_m[side][par];
    if (mp > 0) {
      if (m + mp > cap) {
        wv_qr_traced(e, m, Kt, A);
        const int mc = m < Kt ? m : Kt;
        for (int q = lane; q < mc * mc; q += 64) { const int i = q % mc, j = q / mc; if (i > j) A(i, j) = 0.0; }
        wave_sync();
        m = mc;
      }
      MV Bp = wslot(e.wB[side], par), Et = Eslot(e, side, t);
      const bool root_of_sub = insub && t == u.r0[side];
      // B~_parent diag(E_t, I)^*: the transfer product, then the identity part
      if (kpar > 0)
        wv_mm_f64(mp, kt, kpar, [&](int i, int l) { return Bp(i, l); }, [&](int l, int j) { return Et(j, l); },
                  [&](int i, int j, double v) { A(m + i, j) = v; });
      else
        for (int q = lane; q < mp * kt; q += 64) A(m + q % mp, q / mp) = 0.0;
      for (int q = lane; q < mp * (Kt - kt); q += 64) {
        const int i = q % mp, j = kt + q / mp;
        A(m + i, j) = root_of_sub ? 0.0 : Bp(i, kpar + (j - kt));   // identity part of diag(E_t, I)
      }
      wave_sync();
      fl += fl_gemm(mp, kt, kpar);
      m += mp;
      mrows += mp;
    }
  }
  int mr = 0;
  wt_add(e, WT_W_STACK, tw);
  if (m > 0) {
    wv_qr_traced(e, m, Kt, A);
    mr = m < Kt ? m : Kt;
    for (int q = lane; q < mr * Kt; q += 64) {
      const int i = q % mr, j = q / mr;
      Wt(i, j) = j >= i ? A(i, j) : 0.0;
    }
  }
  if (lane == 0) e.wB_m[side][t] = mr;
  wt_add(e, WT_W_QR, tw);
  count_w(e, W, ST_A5, fl + fl_qr(mrows, Kt));
  wave_sync();
}

// Step 4: nested recompression of cluster c (Section 4, eq. (Qt_nested),
// (hatQt_condensed)): truncated SVD of V~_t B~_t^* (leaf) or V^_t B~_t^*,
// new basis / transfer matrices and R_t = Q_t^* V~_t.  Returns the new rank
// or -1 past the rank cap (one wave).
__device__ int wv_recompress(const DevEnv &e, const Upd &u, const Wv &W, int side, int c) {
  const int lane = lane_id();
  unsigned long long tw = wt_now(e);
  const int root = u.r0[side];
  const int kc = e.k[side][c], K = kc + u.kp;
  WvAlloc al = wv_alloc(e, W);
  int mr, r1 = 0;
  MV Vt;
  double fl = 0.0;
  if (is_leaf(e, c)) {
    mr = e.size[c];
    Vt = al.take(mr, K);
    MV V = leafslot(e, side, c), F = bufrows(e, u.buf[side], c);
    for (int q = lane; q < mr * K; q += 64) {
      const int i = q % mr, j = q / mr;
      Vt(i, j) = j < kc ? V(i, j) : F(i, j - kc);
    }
  } else {
    const int c1 = e.son0[c], c2 = e.son1[c];
    const int rc1 = e.wnewk[side][c1], rc2 = e.wnewk[side][c2];
    r1 = rc1;
    mr = rc1 + rc2;
    Vt = al.take(mr, K);
    for (int sn = 0; sn < 2; ++sn) {
      const int ch = sn == 0 ? c1 : c2, rc = sn == 0 ? rc1 : rc2, off = sn == 0 ? 0 : rc1;
      const int kch = e.k[side][ch];
      MV Rc = wslot(e.wR[side], ch), Ec = Eslot(e, side, ch);
      // [R_ch E_ch, R_ch's update columns]: the transfer product, then a copy
      if (kch > 0)
        wv_mm(e.prec != 0, rc, kc, kch, [&](int i, int l) { return Rc(i, l); }, [&](int l, int j) { return Ec(l, j); },
              [&](int i, int j, double v) { Vt(off + i, j) = v; });
      else
        for (int q = lane; q < rc * kc; q += 64) Vt(off + q % rc, q / rc) = 0.0;
      for (int q = lane; q < rc * (K - kc); q += 64) {
        const int i = q % rc, j = kc + q / rc;
        Vt(off + i, j) = Rc(i, kch + (j - kc));
      }
      fl += fl_gemm(rc, kc, kch);
    }
  }
  wave_sync();
  wt_add(e, WT_RC_BUILD, tw);
  const int mB = e.wB_m[side][c];
  int r = 0;
  bool trans = false;
  MV M{nullptr, 0, 0}, J{nullptr, 0, 0}, Y{nullptr, 0, 0};
  double *qtau = nullptr;
  int qsrc = 0;   // 0: columns of M (or of J), 1: columns of Y, 2: Q times columns of Y^*
  if (mr > 0 && mB > 0) {
    M = al.take(mr, mB);
    wv_gemm(mr, mB, K, 1.0, Vt, mv_t(wslot(e.wB[side], c)), 0.0, M);
    fl += fl_gemm(mr, mB, K);
    wt_add(e, WT_RC_M, tw);
    trans = mB > mr;
    int sweeps, nG;
    const unsigned long long tj = wt_now(e);
    if (!trans && mB > PRECOND_MIN) {
      // Two-stage QR preconditioning: M = Q R, R^* = Q2 R2; the left singular
      // vectors of R2^* (its Jacobi-rotated columns, normalised) times Q are
      // those of M, and the sweeps needed on R2^* are few.
      qtau = al.take(mB, 1).p;
      wv_qr(mr, mB, M, qtau);
      Y = al.take(mB, mB);
      for (int q = lane; q < mB * mB; q += 64) {
        const int i = q % mB, j = q / mB;
        Y(i, j) = i >= j ? M(j, i) : 0.0;
      }
      wave_sync();
      wv_qr(mB, mB, Y, nullptr);
      for (int q = lane; q < mB * mB; q += 64) { const int i = q % mB, j = q / mB; if (i > j) Y(i, j) = 0.0; }
      wave_sync();
      sweeps = wave_jacobi(mB, mB, mv_t(Y), nullptr);
      wv_colnorms_sorted(mB, mB, mv_t(Y), W.sig, W.ord);
      nG = mB;
      qsrc = 2;
      fl += 2.0 * fl_qr(mr, mB) + fl_qr(mB, mB);
    } else if (trans && mr > PRECOND_MIN) {
      // M^* = Q1 R1: the left singular vectors of M are those of R1^*
      const MV Mt = mv_t(M);
      wv_qr(mB, mr, Mt, nullptr);
      Y = al.take(mr, mr);
      for (int q = lane; q < mr * mr; q += 64) {
        const int i = q % mr, j = q / mr;
        Y(i, j) = i >= j ? Mt(j, i) : 0.0;
      }
      wave_sync();
      sweeps = wave_jacobi(mr, mr, Y, nullptr);
      wv_colnorms_sorted(mr, mr, Y, W.sig, W.ord);
      nG = mr;
      qsrc = 1;
      fl += fl_qr(mB, mr);
    } else if (!trans) {
      sweeps = wave_jacobi(mr, mB, M, nullptr);
      wv_colnorms_sorted(mr, mB, M, W.sig, W.ord);
      nG = mB;
    } else {
      // left singular vectors of M = accumulated rotations of M^*
      J = al.take(mr, mr);
      for (int q = lane; q < mr * mr; q += 64) J(q % mr, q / mr) = (q % mr == q / mr) ? 1.0 : 0.0;
      wave_sync();
      MV Mt = mv_t(M);
      sweeps = wave_jacobi(mB, mr, Mt, &J);
      wv_colnorms_sorted(mB, mr, Mt, W.sig, W.ord);
      nG = mr;
    }
    fl += fl_svd(mr, mB);
    wt_add(e, WT_RC_SVD, tw);
    if (e.prof && lane == 0) {
      const int cls = nG <= 8 ? 0 : nG <= 16 ? 1 : nG <= 32 ? 2 : 3;
      atomicAdd(&e.prof[PROF_LEAFSTAGE + 8 + cls], wall_clock64() - tj);
      atomicAdd(&e.prof[PROF_LEAFSTAGE + 12 + cls], 1ull);
      atomicAdd(&e.prof[PROF_STAGE + 12], (unsigned long long)sweeps);
      atomicAdd(&e.prof[PROF_STAGE + 13], 1ull);
      atomicAdd(&e.prof[PROF_STAGE + 14], (unsigned long long)nG);
    }
    // at least the rounding level max(m, n) eps sigma_1 (numerical rank):
    // singular vectors of smaller values are not determined by the data
    const double smax = nG > 0 ? W.sig[W.ord[0]] : 0.0;
    // variable-order weighting: the threshold times q^(depth - level(c)),
    // formed by repeated products (q = 1: unchanged)
    double lsc = 1.0;
    if (e.lvq != 1.0)
      for (int l = e.level[c]; l < e.depth; ++l) lsc *= e.lvq;
    const double tau = fmax(trunc_tau(e, smax) * lsc, (double)(mr > mB ? mr : mB) * 2.220446049250313e-16 * smax);
    for (int j = 0; j < nG; ++j) r += W.sig[W.ord[j]] > tau ? 1 : 0;
    if (r > e.rank_cap) {
      if (lane == 0) { e.err[1] = c; e.err[0] = E_RANK_CAP; }
      wave_sync();
      return -1;
    }
  }
  MV Q = al.take(mr, r > 0 ? r : 1);
  for (int q = lane; q < mr * r; q += 64) {
    const int i = q % mr, j = q / mr;
    const int cc = W.ord[j];
    double v;
    if (qsrc == 2) v = i < mB ? Y(cc, i) / W.sig[cc] : 0.0;   // columns of R2^*, padded
    else if (qsrc == 1) v = Y(i, cc) / W.sig[cc];
    else v = trans ? J(i, cc) : M(i, cc) / W.sig[cc];
    Q(i, j) = v;
  }
  wave_sync();
  if (qsrc == 2) {
    wv_apply_q(mr, mB, M, qtau, Q, r);
    fl += fl_gemm(mr, r, mB);
  }
  wv_gemm(r, K, mr, 1.0, mv_t(Q), Vt, 0.0, wslot(e.wR[side], c), e.prec != 0);   // R_c = Q^* V~_c
  fl += fl_gemm(r, K, mr);
  if (lane == 0) e.wnewk[side][c] = r;
  if (is_leaf(e, c)) {
    MV V = leafslot(e, side, c);
    if (e.prec == 2)   // trial form: leaf bases kept at bfloat16 precision
      for (int q = lane; q < mr * r; q += 64) V(q % mr, q / mr) = round_bf16(Q(q % mr, q / mr));
    else
      for (int q = lane; q < mr * r; q += 64) V(q % mr, q / mr) = Q(q % mr, q / mr);
  } else {
    MV E1 = Eslot(e, side, e.son0[c]), E2 = Eslot(e, side, e.son1[c]);
    const int r2 = mr - r1;
    for (int q = lane; q < r1 * r; q += 64) E1(q % r1, q / r1) = Q(q % r1, q / r1);
    for (int q = lane; q < r2 * r; q += 64) E2(q % r2, q / r2) = Q(r1 + q % r2, q / r2);
  }
  wave_sync();
  if (c == root && e.parent[c] >= 0) {
    // E_{t0} <- R_{t0} [E_{t0}; 0]
    const int kpar = e.k[side][e.parent[c]];
    MV T = al.take(r, kpar);
    MV Ec = Eslot(e, side, c);
    wv_gemm(r, kpar, kc, 1.0, wslot(e.wR[side], c), Ec, 0.0, T, e.prec != 0);
    for (int q = lane; q < r * kpar; q += 64) Ec(q % r, q / r) = T(q % r, q / r);
    fl += fl_gemm(r, kpar, kc);
  }
  count_w(e, W, ST_A6, fl);
  // transfers of the sons read (inner) and the new basis / transfers written
  bytes_w(e, ST_A6, is_leaf(e, c) ? 8.0 * mr * r
                                  : 8.0 * ((double)(e.k[side][e.son0[c]] + e.k[side][e.son1[c]]) * kc + (double)mr * r));
  wave_sync();
  wt_add(e, WT_RC_OUT, tw);
  return r;
}

// Step 5: coupling of an admissible leaf touching the subtrees,
// S_b <- R_t S~_b R_s^* (identity factor outside the subtrees).
__device__ void wv_coupling(const DevEnv &e, const Upd &u, const Wv &W, int b) {
  const int lane = lane_id();
  unsigned long long tw = wt_now(e);
  const SExt St = sext(e, u, b);
  const int t = e.brow[b], s = e.bcol[b];
  WvAlloc al = wv_alloc(e, W);
  const int rows = St.tin ? e.wnewk[0][t] : St.kt;
  MV P = al.take(rows, St.Ks);
  double fl = 0.0;
  const bool f32 = e.prec != 0;
  if (St.tin) {
    MV Rt = wslot(e.wR[0], t);
    if (St.Kt > 0)
      wv_mm(f32, rows, St.Ks, St.Kt, [&](int i, int l) { return Rt(i, l); }, [&](int l, int j) { return St(l, j); },
            [&](int i, int j, double v) { P(i, j) = v; });
    else
      for (int q = lane; q < rows * St.Ks; q += 64) P(q % rows, q / rows) = 0.0;
    fl += fl_gemm(rows, St.Ks, St.Kt);
  } else {
    for (int q = lane; q < rows * St.Ks; q += 64) P(q % rows, q / rows) = St(q % rows, q / rows);
  }
  wave_sync();
  MV Sd = Sslot(e, b);
  if (St.sin) {
    const int rs = e.wnewk[1][s];
    wv_gemm(rows, rs, St.Ks, 1.0, P, mv_t(wslot(e.wR[1], s)), 0.0, Sd, f32);
    fl += fl_gemm(rows, rs, St.Ks);
  } else {
    for (int q = lane; q < rows * St.Ks; q += 64) Sd(q % rows, q / rows) = P(q % rows, q / rows);
  }
  count_w(e, W, ST_A7, fl);
  bytes_w(e, ST_A7, 8.0 * ((double)St.kt * St.ks + (double)rows * (St.sin ? e.wnewk[1][s] : St.Ks)));
  wave_sync();
  wt_add(e, WT_CPL, tw);
}

// R-factor of a predecessor's basis after E_{t0} changed (one wave).
// R-factor of the basis of c from its sons (rho_c = R of [rho_c1 E_c1;
// rho_c2 E_c2]).  The son vs, if it is one, is the root of a subtree just
// recompressed whose new rank vr is not committed yet: its basis is
// orthonormal, so its block is E_vs itself.
__device__ void wv_refresh_rho(const DevEnv &e, const Wv &W, int side, int c, int vs, int vr) {
  const int lane = lane_id();
  unsigned long long tw = wt_now(e);
  wc_add(e, WC_REFRESH, 1);
  const int kc = e.k[side][c];
  const int c1 = e.son0[c], c2 = e.son1[c];
  const int m1 = c1 == vs ? vr : e.rho_m[side][c1], m2 = c2 == vs ? vr : e.rho_m[side][c2];
  WvAlloc al = wv_alloc(e, W);
  MV A = al.take(m1 + m2, kc);
  for (int sn = 0; sn < 2; ++sn) {
    const int cs = sn == 0 ? c1 : c2, ms = sn == 0 ? m1 : m2, off = sn == 0 ? 0 : m1;
    const MV Es = Eslot(e, side, cs);
    if (cs == vs) {
      for (int q = lane; q < ms * kc; q += 64) A(off + q % ms, q / ms) = Es(q % ms, q / ms);
      wave_sync();
    } else {
      wv_gemm(ms, kc, e.k[side][cs], 1.0, rhoslot(e, side, cs), Es, 0.0, mv_at(A, off, 0));
    }
  }
  const int m = m1 + m2;
  wv_qr(m, kc, A, nullptr);
  const int mr = m < kc ? m : kc;
  MV R = rhoslot(e, side, c);
  for (int q = lane; q < mr * kc; q += 64) {
    const int i = q % mr, j = q / mr;
    R(i, j) = j >= i ? A(i, j) : 0.0;
  }
  if (lane == 0) e.rho_m[side][c] = mr;
  count_w(e, W, ST_A8, fl_qr(m, kc) + (c1 == vs ? 0.0 : fl_gemm(m1, kc, e.k[side][c1])) +
                           (c2 == vs ? 0.0 : fl_gemm(m2, kc, e.k[side][c2])));
  bytes_w(e, ST_A8, 8.0 * ((double)e.k[side][c1] + e.k[side][c2]) * kc);   // the sons' transfers
  wave_sync();
  wt_add(e, WT_REFRESH, tw);
}

__device__ __forceinline__ void prof_stage(const DevEnv &e, int stage, unsigned long long &t,
                                           bool leaf = false) {
  if (e.prof && threadIdx.x == 0) {
    const unsigned long long now = wall_clock64();
    e.prof[PROF_STAGE + stage] += now - t;
    if (leaf) e.prof[PROF_LEAFSTAGE + stage] += now - t;
    t = now;
  }
}

// Number of descendants of r at level lv (0 above r's level or below the leaves).
__device__ __forceinline__ int nlevel(const DevEnv &e, int r, int lv) {
  return lv < e.level[r] ? 0 : dhi(e, r, lv) - dlo(e, r, lv);
}

// Ancestor of c at level lv <= level(c).
__device__ __forceinline__ int ancestor(const DevEnv &e, int c, int lv) {
  while (e.level[c] > lv) c = e.parent[c];
  return c;
}

__device__ void task_addlr(const DevEnv &e, const Lds &L, double *lds, int b0, int bx, int by) {
  unsigned long long tstage = wall_clock64();
  const unsigned long long tstart = tstage;
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
  const Wv W = wave_areas(lds, e);
  const int lv0[2] = {e.level[u.r0[0]], e.level[u.r0[1]]};
  const int lvmin = lv0[0] < lv0[1] ? lv0[0] : lv0[1];
  const bool leafupd = is_leaf(e, u.r0[0]);
  // --- steps 2/3, first part: block rows of the weights of the predecessors
  // above both subtrees.  They read only data outside the subtrees, so they
  // run concurrently with each other and with step 1.
  const int npath = lvmin;
  for (int q = W.w; q < 2 * npath; q += NWAVE) {
    const int side = q < npath ? 0 : 1, lv = q < npath ? q : q - npath;
    wv_weight(e, u, W, side, ancestor(e, u.r0[side], lv), false, W_ROWS);
  }
  // --- step 1: R-factors of the extended bases, bottom-up, clusters of a level concurrently
  for (int lv = e.nlev - 1; lv >= lvmin; --lv) {
    const int n0 = nlevel(e, u.r0[0], lv), n1 = nlevel(e, u.r0[1], lv);
    for (int q = W.w; q < n0 + n1; q += NWAVE) {
      const int side = q < n0 ? 0 : 1;
      const int c = side == 0 ? dlo(e, u.r0[0], lv) + q : dlo(e, u.r0[1], lv) + (q - n0);
      wv_rfactor(e, u, W, side, c);
    }
    __syncthreads();
  }
  prof_stage(e, 1, tstage, leafupd);
  // --- steps 2/3, second part: the chain root -> parent(t0) adds the parent
  // rows (one wave per side), then the remaining levels top-down
  if (W.w < 2) {
    const int side = W.w;
    for (int lv = 1; lv < npath; ++lv) wv_weight(e, u, W, side, ancestor(e, u.r0[side], lv), false, W_CHAIN);
  }
  __syncthreads();
  for (int lv = npath; lv < e.nlev; ++lv) {
    int cnt[2];
    for (int side = 0; side < 2; ++side) cnt[side] = lv < lv0[side] ? 1 : nlevel(e, u.r0[side], lv);
    for (int q = W.w; q < cnt[0] + cnt[1]; q += NWAVE) {
      const int side = q < cnt[0] ? 0 : 1;
      const int qq = side == 0 ? q : q - cnt[0];
      if (lv < lv0[side]) wv_weight(e, u, W, side, ancestor(e, u.r0[side], lv), false, W_FULL);
      else wv_weight(e, u, W, side, dlo(e, u.r0[side], lv) + qq, true, W_FULL);
    }
    __syncthreads();
  }
  prof_stage(e, 3, tstage, leafupd);
  // --- step 4: nested recompression, bottom-up
  for (int lv = e.nlev - 1; lv >= lvmin; --lv) {
    const int n0 = nlevel(e, u.r0[0], lv), n1 = nlevel(e, u.r0[1], lv);
    for (int q = W.w; q < n0 + n1; q += NWAVE) {
      const int side = q < n0 ? 0 : 1;
      const int c = side == 0 ? dlo(e, u.r0[0], lv) + q : dlo(e, u.r0[1], lv) + (q - n0);
      wv_recompress(e, u, W, side, c);
    }
    __syncthreads();
    if (e.err[0] != 0) return;
  }
  prof_stage(e, 4, tstage, leafupd);
  // --- step 6, first part: R-factors on the paths root -> parent(t0) and
  // root -> parent(s0) (one wave per side).  They read only the recompressed
  // subtree roots and the bases above them, so they run while the other
  // waves (and these, afterwards) update the couplings and nearfield blocks.
  if (W.w < 2) {
    const int side = W.w, root = u.r0[side];
    for (int c = e.parent[root]; c >= 0; c = e.parent[c]) wv_refresh_rho(e, W, side, c, root, e.wnewk[side][root]);
  }
  // --- step 5: couplings of every admissible leaf touching the subtrees,
  // assigned greedily to the least loaded wave (waves 0 and 1 start with the
  // path refreshes, counted as one item each)
  {
    int load[NWAVE];
    for (int w = 0; w < NWAVE; ++w) load[w] = w < 2 ? lv0[w] : 0;
    for (int side = 0; side < 2; ++side) {
      const int root = u.r0[side];
      const int *ptr = side == 0 ? e.rowptr : e.colptr;
      const int *idx = side == 0 ? e.rowidx : e.colidx;
      for (int lv = lv0[side]; lv < e.nlev; ++lv) {
        const int lo = dlo(e, root, lv), hi = lo + nlevel(e, root, lv);
        for (int c = lo; c < hi; ++c) {
          for (int p = ptr[c]; p < ptr[c + 1]; ++p) {
            const int b = idx[p];
            if (side == 1 && in_sub(e, u.r0[0], e.brow[b])) continue;
            int wmin = 0;
            for (int w = 1; w < NWAVE; ++w) wmin = load[w] < load[wmin] ? w : wmin;
            ++load[wmin];
            if (wmin == W.w) wv_coupling(e, u, W, b);
          }
        }
      }
    }
    __syncthreads();
  }
  prof_stage(e, 5, tstage, leafupd);
  // --- step 7: inadmissible leaves inside b0 receive X|_t Y|_s^*
  {
    int q = 0;
    const int root = u.r0[0];
    for (int lv = lv0[0]; lv < e.nlev; ++lv) {
      const int lo = dlo(e, root, lv), hi = lo + nlevel(e, root, lv);
      for (int c = lo; c < hi; ++c) {
        if (!is_leaf(e, c)) continue;
        for (int p = e.nrowptr[c]; p < e.nrowptr[c + 1]; ++p) {
          const int b = e.nrowidx[p];
          const int s = e.bcol[b];
          if (!in_sub(e, u.r0[1], s)) continue;
          if (q % NWAVE == W.w) {
            wv_gemm(e.size[c], e.size[s], u.kp, 1.0, bufrows(e, u.buf[0], c), mv_t(bufrows(e, u.buf[1], s)),
                    1.0, Nslot(e, b));
            count_w(e, W, ST_A9, fl_gemm(e.size[c], e.size[s], u.kp));
            bytes_w(e, ST_A9, 16.0 * e.size[c] * e.size[s]);
          }
          ++q;
        }
      }
    }
    __syncthreads();
  }
  prof_stage(e, 6, tstage, leafupd);
  // --- step 6: commit ranks, identity R-factors of the new bases, refresh the paths
  for (int side = 0; side < 2; ++side) {
    const int root = u.r0[side];
    for (int lv = lv0[side]; lv < e.nlev; ++lv) {
      const int lo = dlo(e, root, lv), hi = lo + nlevel(e, root, lv);
      for (int c = lo; c < hi; ++c) {
        const int r = e.wnewk[side][c];
        MV R = rhoslot(e, side, c);
        for (int q = threadIdx.x; q < r * r; q += blockDim.x) R(q % r, q / r) = (q % r == q / r) ? 1.0 : 0.0;
        if (threadIdx.x == 0) { e.k[side][c] = r; e.rho_m[side][c] = r; }
      }
    }
  }
  __syncthreads();
  prof_stage(e, 7, tstage, leafupd);
  if (e.prof && threadIdx.x == 0) {
    const int lv = lv0[0] < 15 ? lv0[0] : 15;
    e.prof[PROF_LEVEL + lv] += wall_clock64() - tstart;
    e.prof[PROF_LEVEL + 16 + lv] += 1;
  }
}

// OP_ADDLR (one local update with the factors in buffers i1, i2) and
// OP_ADDLR_ACC: the temporaries T0..T(np-1) of an admissible product target
// (each the truncated sum of the son-pair products, on the rows of t and r)
// enter the matrix by local updates, one each in order (e.acc == 0), or
// accumulated: consecutive temporaries are concatenated into the update
// buffers while the total rank stays within KPMAX, one update per group.
// One call site of task_addlr for both (a second inlined copy of the update
// enlarges the interpreter's stack frame).
__device__ void task_addlr_tk(const DevEnv &e, const Lds &L, double *lds, const Task &tk) {
  const int b0 = tk.i[0];
  const bool temps = tk.op == OP_ADDLR_ACC;
  const int np = temps ? tk.i[1] : 1;
  const int t = e.brow[b0], r = e.bcol[b0];
  for (int p = 0; p < np;) {
    int q = p + 1;
    int bx = temps ? B_T0U + 2 * p : tk.i[1], by = temps ? B_T0V + 2 * p : tk.i[2];
    if (temps && e.acc) {
      int kt = e.bcols[B_T0U + 2 * p];
      while (q < np && kt + e.bcols[B_T0U + 2 * q] <= KPMAX) kt += e.bcols[B_T0U + 2 * q++];
      if (q > p + 1) {
        int c0 = 0;
        for (int j = p; j < q; ++j) {
          const int kj = e.bcols[B_T0U + 2 * j];
          for (int side = 0; side < 2; ++side) {
            const int c = side == 0 ? t : r;
            const MV src = bufrows(e, (side == 0 ? B_T0U : B_T0V) + 2 * j, c);
            const MV dst = bufrows(e, side == 0 ? B_U : B_V, c);
            const int rows = e.size[c];
            for (int x = threadIdx.x; x < rows * kj; x += blockDim.x)
              dst(x % rows, c0 + x / rows) = src(x % rows, x / rows);
          }
          c0 += kj;
        }
        if (threadIdx.x == 0) { e.bcols[B_U] = kt; e.bcols[B_V] = kt; }
        __syncthreads();
        bx = B_U;
        by = B_V;
      }
    }
    task_addlr(e, L, lds, b0, bx, by);
    p = q;
    if (p < np) {
      __syncthreads();
      if (e.err[0] != 0) return;
    }
  }
}

// ====================================================== products with H^2
// Expanded basis of cluster t (through eq. (nested)) into buffer rows of t.
__device__ void task_expand(const DevEnv &e, int side, int t, int bo) {
  const int kt = e.k[side][t];
  MV out = bufrows(e, bo, t);
  if (kt == 0) {
    // (nothing to expand)
  } else if (is_leaf(e, t)) {
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
// b = (t, s).  A leaf block of two leaf clusters is staged into LDS and
// evaluated there; other blocks use the forward transformation, couplings,
// backward transformation and nearfield products, one wave per cluster.
__device__ void bapply_leaf(const DevEnv &e, const Lds &L, int b, int trans, int bin, int bout,
                            double alpha, double beta, int m) {
  const int t = e.brow[b], s = e.bcol[b];
  const int nt = e.size[t], ns = e.size[s];
  const int nsrc = trans ? nt : ns, ndst = trans ? ns : nt;
  const int src = trans ? t : s, dst = trans ? s : t;
  MV x = mv_col(L.W0, LS);                 // nsrc x m
  MV in = bufrows(e, bin, src), out = bufrows(e, bout, dst);
  double fl;
  if (e.bkind[b] == 2) {
    MV N = mv_col(L.W1, LS);               // nt x ns
    MV Ns = Nslot(e, b);
    for (Walk2 w(threadIdx.x, blockDim.x, nsrc); w.j < m; w.next()) x(w.i, w.j) = in(w.i, w.j);
    for (Walk2 w(threadIdx.x, blockDim.x, nt); w.j < ns; w.next()) N(w.i, w.j) = Ns(w.i, w.j);
    __syncthreads();
    for (Walk2 w(threadIdx.x, blockDim.x, ndst); w.j < m; w.next()) {
      double acc = 0.0;
      if (!trans) { for (int l = 0; l < ns; ++l) acc = fma(N(w.i, l), x(l, w.j), acc); }
      else { for (int l = 0; l < nt; ++l) acc = fma(N(l, w.i), x(l, w.j), acc); }
      out(w.i, w.j) = (beta == 0.0 ? 0.0 : beta * out(w.i, w.j)) + alpha * acc;
    }
    fl = 2.0 * nt * ns * m;
  } else {
    const int kt = e.k[0][t], ks = e.k[1][s];
    const int ksrc = trans ? kt : ks, kdst = trans ? ks : kt;
    MV Vs = mv_col(L.W1, LS), Vd = mv_col(L.W1 + LS * KC, LS);   // source / destination bases
    MV S = mv_col(L.W2, KC);
    MV xh = mv_col(L.W2 + KC * KC, KC), yh = mv_col(L.W0 + LS * BC, KC);   // k x m (m <= BC)
    MV Bs = leafslot(e, trans ? 0 : 1, src), Bd = leafslot(e, trans ? 1 : 0, dst), Sg = Sslot(e, b);
    for (Walk2 w(threadIdx.x, blockDim.x, nsrc); w.j < m; w.next()) x(w.i, w.j) = in(w.i, w.j);
    if (ksrc > 0) for (Walk2 w(threadIdx.x, blockDim.x, nsrc); w.j < ksrc; w.next()) Vs(w.i, w.j) = Bs(w.i, w.j);
    if (kdst > 0) for (Walk2 w(threadIdx.x, blockDim.x, ndst); w.j < kdst; w.next()) Vd(w.i, w.j) = Bd(w.i, w.j);
    if (kt > 0) for (Walk2 w(threadIdx.x, blockDim.x, kt); w.j < ks; w.next()) S(w.i, w.j) = Sg(w.i, w.j);
    __syncthreads();
    if (ksrc > 0) for (Walk2 w(threadIdx.x, blockDim.x, ksrc); w.j < m; w.next()) {
      double acc = 0.0;
      for (int l = 0; l < nsrc; ++l) acc = fma(Vs(l, w.i), x(l, w.j), acc);
      xh(w.i, w.j) = acc;
    }
    __syncthreads();
    if (kdst > 0) for (Walk2 w(threadIdx.x, blockDim.x, kdst); w.j < m; w.next()) {
      double acc = 0.0;
      if (!trans) { for (int l = 0; l < ks; ++l) acc = fma(S(w.i, l), xh(l, w.j), acc); }
      else { for (int l = 0; l < kt; ++l) acc = fma(S(l, w.i), xh(l, w.j), acc); }
      yh(w.i, w.j) = acc;
    }
    __syncthreads();
    for (Walk2 w(threadIdx.x, blockDim.x, ndst); w.j < m; w.next()) {
      double acc = 0.0;
      for (int l = 0; l < kdst; ++l) acc = fma(Vd(w.i, l), yh(l, w.j), acc);
      out(w.i, w.j) = (beta == 0.0 ? 0.0 : beta * out(w.i, w.j)) + alpha * acc;
    }
    fl = 2.0 * m * ((double)nsrc * ksrc + (double)kt * ks + (double)ndst * kdst);
  }
  count(e, fl);
  if (threadIdx.x == 0) e.bcols[bout] = m;
  __syncthreads();
}

__device__ void task_bapply(const DevEnv &e, const Lds &L, int b, int trans, int bin, int bout,
                            double alpha, double beta) {
  const int m = e.bcols[bin];
  const int t = e.brow[b], s = e.bcol[b];
  if (m == 0) {   // no columns: nothing to compute (happens while ranks are still zero)
    if (threadIdx.x == 0) e.bcols[bout] = 0;
    __syncthreads();
    return;
  }
  if (e.bkind[b] != 0 && is_leaf(e, t) && is_leaf(e, s)) {
    bapply_leaf(e, L, b, trans, bin, bout, alpha, beta, m);
    return;
  }
  const int sr = trans ? t : s, dr = trans ? s : t;
  const int ss = trans ? 0 : 1, ds = 1 - ss;
  const int lane = lane_id(), wv = wave_id();
  double fl = 0.0;   // counted by lane 0 of each wave
  // For a subdivided block (t, s) the leaves below pair sons of t with sons
  // of s (a leaf cluster stands for itself), so the forward transformation
  // of a source root with sons and the coupling sum of a destination root
  // with sons are never used and are skipped.  A root that is a leaf (the
  // other root then has sons, in unbalanced trees) is kept.
  const int inner = e.bkind[b] == 0 ? 1 : 0;
  const int top_s = inner && !is_leaf(e, sr) ? 1 : 0, top_d = inner && !is_leaf(e, dr) ? 1 : 0;
  // forward transformation over the source subtree
  for (int lv = e.nlev - 1; lv >= e.level[sr] + top_s; --lv) {
    const int lo = dlo(e, sr, lv), hi = lo + nlevel(e, sr, lv);
    for (int c = lo + wv; c < hi; c += NWAVE) {
      const int kc = e.k[ss][c];
      MV xc = xhslot(e.xh, c);
      if (is_leaf(e, c)) {
        MV V = leafslot(e, ss, c), x = bufrows(e, bin, c);
        const int nc = e.size[c];
        if (kc > 0) for (Walk2 w(lane, 64, kc); w.j < m; w.next()) {
          double acc = 0.0;
          acc = dotc<8>(0, nc, [&](int l) { return V(l, w.i); }, [&](int l) { return x(l, w.j); }, acc);
          xc(w.i, w.j) = acc;
        }
        if (lane == 0) fl += 2.0 * nc * kc * m;
      } else {
        const int c1 = e.son0[c], c2 = e.son1[c];
        const int k1 = e.k[ss][c1], k2 = e.k[ss][c2];
        MV E1 = Eslot(e, ss, c1), E2 = Eslot(e, ss, c2), x1 = xhslot(e.xh, c1), x2 = xhslot(e.xh, c2);
        if (kc > 0) for (Walk2 w(lane, 64, kc); w.j < m; w.next()) {
          double acc = 0.0;
          acc = dotc(0, k1, [&](int l) { return E1(l, w.i); }, [&](int l) { return x1(l, w.j); }, acc);
          acc = dotc(0, k2, [&](int l) { return E2(l, w.i); }, [&](int l) { return x2(l, w.j); }, acc);
          xc(w.i, w.j) = acc;
        }
        if (lane == 0) fl += 2.0 * (k1 + k2) * kc * m;
      }
    }
    __syncthreads();
  }
  // destination subtree, top-down, one pass per level: the coupling sum
  // yh_c = sum_b S_b xh_o + E_c yh_parent, and for a leaf right away the rows
  // out_c = beta out_c + alpha (V_c yh_c + sum_near N_b x_o)  (every row of
  // the destination belongs to exactly one leaf)
  const int *ptr = trans ? e.colptr : e.rowptr;
  const int *idx = trans ? e.colidx : e.rowidx;
  const int *nptr = trans ? e.ncolptr : e.nrowptr;
  const int *nidx = trans ? e.ncolidx : e.nrowidx;
  for (int lv = e.level[dr] + top_d; lv < e.nlev; ++lv) {
    const int lo = dlo(e, dr, lv), hi = lo + nlevel(e, dr, lv);
    for (int c = lo + wv; c < hi; c += NWAVE) {
      const int kc = e.k[ds][c];
      MV yc = xhslot(e.yh, c);
      if (kc > 0) {
        for (Walk2 w(lane, 64, kc); w.j < m; w.next()) yc(w.i, w.j) = 0.0;
        for (int p = ptr[c]; p < ptr[c + 1]; ++p) {
          const int bb = idx[p];
          const int o = trans ? e.brow[bb] : e.bcol[bb];
          if (!in_sub(e, sr, o)) continue;
          MV S = Sslot(e, bb), xo = xhslot(e.xh, o);
          const int ko = e.k[ss][o];
          for (Walk2 w(lane, 64, kc); w.j < m; w.next()) {
            double acc = yc(w.i, w.j);
            if (!trans) { acc = dotc(0, ko, [&](int l) { return S(w.i, l); }, [&](int l) { return xo(l, w.j); }, acc); }
            else { acc = dotc(0, ko, [&](int l) { return S(l, w.i); }, [&](int l) { return xo(l, w.j); }, acc); }
            yc(w.i, w.j) = acc;
          }
          if (lane == 0) fl += 2.0 * kc * ko * m;
        }
        if (lv > e.level[dr] + top_d) {
          const int pc = e.parent[c];
          const int kp = e.k[ds][pc];
          MV Ec = Eslot(e, ds, c), yp = xhslot(e.yh, pc);
          for (Walk2 w(lane, 64, kc); w.j < m; w.next()) {
            double acc = yc(w.i, w.j);
            acc = dotc(0, kp, [&](int l) { return Ec(w.i, l); }, [&](int l) { return yp(l, w.j); }, acc);
            yc(w.i, w.j) = acc;
          }
          if (lane == 0) fl += 2.0 * kc * kp * m;
        }
      }
      if (is_leaf(e, c)) {
        wave_sync();
        const int nc = e.size[c];
        MV V = leafslot(e, ds, c), oc = bufrows(e, bout, c);
        for (Walk2 w(lane, 64, nc); w.j < m; w.next()) {
          double acc = 0.0;
          acc = dotc(0, kc, [&](int l) { return V(w.i, l); }, [&](int l) { return yc(l, w.j); }, acc);
          for (int p = nptr[c]; p < nptr[c + 1]; ++p) {
            const int bb = nidx[p];
            const int o = trans ? e.brow[bb] : e.bcol[bb];
            if (!in_sub(e, sr, o)) continue;
            MV N = Nslot(e, bb), xo = bufrows(e, bin, o);
            const int no = e.size[o];
            if (!trans) { acc = dotc<8>(0, no, [&](int l) { return N(w.i, l); }, [&](int l) { return xo(l, w.j); }, acc); }
            else { acc = dotc<8>(0, no, [&](int l) { return N(l, w.i); }, [&](int l) { return xo(l, w.j); }, acc); }
          }
          oc(w.i, w.j) = (beta == 0.0 ? 0.0 : beta * oc(w.i, w.j)) + alpha * acc;
        }
        if (lane == 0) {
          fl += 2.0 * nc * kc * m;
          for (int p = nptr[c]; p < nptr[c + 1]; ++p) {
            const int o = trans ? e.brow[nidx[p]] : e.bcol[nidx[p]];
            if (in_sub(e, sr, o)) fl += 2.0 * nc * e.size[o] * m;
          }
        }
      }
    }
    __syncthreads();
  }
  if (lane == 0 && e.flops) e.flops[1 + wv] += fl;
  __syncthreads();
  if (threadIdx.x == 0) e.bcols[bout] = m;
  __syncthreads();
}

// ------------------------------------------------------ H^2 substitution
// Vector substitution L x = b (trans = 0) or L^* x = b (trans = 1) with the
// factor in H^2 form, following the recursion of Section 3 (solve the first
// son, subtract the block (c2, c1) applied to its solution, solve the second
// son).  The block products are not formed one by one: the forward
// transformation xh_s = W_s^* x|_s of every solved cluster is computed once
// (leaf, then transfer matrices upwards) and reused by every block that
// needs it, and coupling contributions S_b xh_s to an unsolved cluster t are
// summed in yh_t and moved to the sons with the transfer matrices just before
// they are solved.  The sums are the same as in the block-by-block form, in
// another association order.  trans = 0: yh in the row basis (side 0), xh in
// the column basis (side 1); trans = 1: the roles are exchanged.

__device__ void task_sv_zero(const DevEnv &e, int c, int bi, int trans) {
  const int side = trans ? 1 : 0, m = e.bcols[bi];
  const int wv = wave_id(), lane = lane_id();
  for (int lv = e.level[c]; lv < e.nlev; ++lv) {
    const int lo = dlo(e, c, lv), hi = lo + nlevel(e, c, lv);
    for (int t = lo + wv; t < hi; t += num_waves()) {
      const int kt = e.k[side][t];
      MV y = xhslot(e.yh, t);
      if (kt > 0)   // (Walk2 needs a non-empty row range)
        for (Walk2 w(lane, 64, kt); w.j < m; w.next()) y(w.i, w.j) = 0.0;
    }
  }
  __syncthreads();
}

__device__ void task_sv_push(const DevEnv &e, int c, int bi, int trans) {
  const int side = trans ? 1 : 0, m = e.bcols[bi];
  const int kc = e.k[side][c];
  const int wv = wave_id(), lane = lane_id();
  if (kc > 0 && wv < 2) {
    const int s = wv == 0 ? e.son0[c] : e.son1[c];
    const int ks = e.k[side][s];
    MV E = Eslot(e, side, s), yp = xhslot(e.yh, c), ys = xhslot(e.yh, s);
    if (ks > 0) for (Walk2 w(lane, 64, ks); w.j < m; w.next()) {
      double acc = ys(w.i, w.j);
      acc = dotc(0, kc, [&](int l) { return E(w.i, l); }, [&](int l) { return yp(l, w.j); }, acc);
      ys(w.i, w.j) = acc;
    }
    if (lane == 0 && e.flops) e.flops[1 + wv] += 2.0 * ks * kc * m;
  }
  __syncthreads();
}

__device__ void task_sv_leaf(const DevEnv &e, int bcc, int bi, int trans) {
  const int c = e.brow[bcc];
  const int side = trans ? 1 : 0, oside = 1 - side, m = e.bcols[bi];
  const int nc = e.size[c], kc = e.k[side][c], ko = e.k[oside][c];
  MV w = bufrows(e, bi, c);
  if (kc > 0) {
    // w -= V_c yh_c (backward transformation of the coupling sums)
    MV V = leafslot(e, side, c), y = xhslot(e.yh, c);
    for (Walk2 q(threadIdx.x, blockDim.x, nc); q.j < m; q.next()) {
      double acc = 0.0;
      acc = dotc(0, kc, [&](int l) { return V(q.i, l); }, [&](int l) { return y(l, q.j); }, acc);
      w(q.i, q.j) -= acc;
    }
    __syncthreads();
  }
  wg_trsv_lower(nc, m, Nslot(e, bcc), w, trans);
  if (ko > 0) {
    // xh_c = W_c^* x|_c
    MV Wb = leafslot(e, oside, c), x = xhslot(e.xh, c);
    for (Walk2 q(threadIdx.x, blockDim.x, ko); q.j < m; q.next()) {
      double acc = 0.0;
      acc = dotc<8>(0, nc, [&](int l) { return Wb(l, q.i); }, [&](int l) { return w(l, q.j); }, acc);
      x(q.i, q.j) = acc;
    }
  }
  count(e, 2.0 * nc * (kc + ko) * m + (double)nc * nc * m);
  __syncthreads();
}

__device__ void task_sv_cross(const DevEnv &e, const int *aux, int off, int ng, int bi, int trans) {
  const int m = e.bcols[bi];
  const int side = trans ? 1 : 0, oside = 1 - side;
  const int wv = wave_id(), lane = lane_id();
  double fl = 0.0;
  // one group per updated cluster t (so no two waves write the same data)
  for (int g = wv; g < ng; g += num_waves()) {
    const int *gp = aux + aux[off + g];
    const int t = gp[0], cnt = gp[1];
    const int kt = e.k[side][t];
    for (int j = 0; j < cnt; ++j) {
      const int b = gp[2 + j];
      const int o = trans ? e.brow[b] : e.bcol[b];
      if (e.bkind[b] == 1) {
        const int ko = e.k[oside][o];
        if (kt == 0 || ko == 0) continue;
        MV S = Sslot(e, b), x = xhslot(e.xh, o), y = xhslot(e.yh, t);
        for (Walk2 w(lane, 64, kt); w.j < m; w.next()) {
          double acc = y(w.i, w.j);
          if (!trans) { acc = dotc(0, ko, [&](int l) { return S(w.i, l); }, [&](int l) { return x(l, w.j); }, acc); }
          else { acc = dotc(0, ko, [&](int l) { return S(l, w.i); }, [&](int l) { return x(l, w.j); }, acc); }
          y(w.i, w.j) = acc;
        }
        fl += 2.0 * kt * ko * m;
      } else {
        const int nt = e.size[t], no = e.size[o];
        MV N = Nslot(e, b), xo = bufrows(e, bi, o), wt = bufrows(e, bi, t);
        for (Walk2 w(lane, 64, nt); w.j < m; w.next()) {
          double acc = 0.0;
          if (!trans) { acc = dotc<8>(0, no, [&](int l) { return N(w.i, l); }, [&](int l) { return xo(l, w.j); }, acc); }
          else { acc = dotc<8>(0, no, [&](int l) { return N(l, w.i); }, [&](int l) { return xo(l, w.j); }, acc); }
          wt(w.i, w.j) -= acc;
        }
        fl += 2.0 * nt * no * m;
      }
    }
  }
  if (lane == 0 && e.flops) e.flops[1 + wv] += fl;
  __syncthreads();
}

__device__ void task_sv_up(const DevEnv &e, int c, int bi, int trans) {
  const int oside = trans ? 0 : 1, m = e.bcols[bi];
  const int kc = e.k[oside][c];
  if (kc > 0) {
    const int c1 = e.son0[c], c2 = e.son1[c];
    const int k1 = e.k[oside][c1], k2 = e.k[oside][c2];
    MV E1 = Eslot(e, oside, c1), E2 = Eslot(e, oside, c2);
    MV x1 = xhslot(e.xh, c1), x2 = xhslot(e.xh, c2), xc = xhslot(e.xh, c);
    for (Walk2 w(threadIdx.x, blockDim.x, kc); w.j < m; w.next()) {
      double acc = 0.0;
      acc = dotc(0, k1, [&](int l) { return E1(l, w.i); }, [&](int l) { return x1(l, w.j); }, acc);
      acc = dotc(0, k2, [&](int l) { return E2(l, w.i); }, [&](int l) { return x2(l, w.j); }, acc);
      xc(w.i, w.j) = acc;
    }
    count(e, 2.0 * (k1 + k2) * kc * m);
  }
  __syncthreads();
}

// out|_cl = alpha in|_cl op(S_b)
__device__ void task_rmul_s(const DevEnv &e, int bin, int bout, int b, int transS, int cl, double alpha) {
  const int kt = e.k[0][e.brow[b]], ks = e.k[1][e.bcol[b]];
  const int kin = transS ? ks : kt, kout = transS ? kt : ks;
  if (kout == 0) {
    if (threadIdx.x == 0) e.bcols[bout] = 0;
    __syncthreads();
    return;
  }
  MV S = Sslot(e, b);
  MV Sop = transS ? mv_t(S) : S;
  wg_gemm(e.size[cl], kout, kin, alpha, bufrows(e, bin, cl), Sop, 0.0, bufrows(e, bout, cl));
  count(e, fl_gemm(e.size[cl], kout, kin));
  if (threadIdx.x == 0) e.bcols[bout] = kout;
  __syncthreads();
}

__device__ void task_copy_near(const DevEnv &e, int b, int bout, int trans, double alpha) {
  const int t = e.brow[b], s = e.bcol[b];
  MV N = Nslot(e, b);
  MV out = bufrows(e, bout, trans ? s : t);
  const int mt = e.size[t], ns = e.size[s];
  for (int q = threadIdx.x; q < mt * ns; q += blockDim.x) {
    const int i = q % mt, j = q / mt;
    if (trans) out(j, i) = alpha * N(i, j);
    else out(i, j) = alpha * N(i, j);
  }
  if (threadIdx.x == 0) e.bcols[bout] = trans ? mt : ns;
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
  if (e.bcols[bu] == 0) return;   // rank-0 contribution
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
__device__ void task_temp_add_wg(const DevEnv &e, const Lds &L, const Task &tk) {
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

// Truncated addition of a product contribution to a low-rank temporary
// (Section 6): [TU U] [TV V]^* = Qa (Ra Rb^*) Qb^*, SVD of the small core
// C = Ra Rb^*, truncation, TU <- Qa U_r Sigma_r, TV <- Qb W_r.  Wave-level
// version: the two QRs run on waves 0 and 1, the core SVD (one-sided Jacobi
// with the rotations accumulated) on wave 0, and the reflectors are applied
// only to the r kept columns.  Temporaries too tall for the wave work areas
// use the workgroup version.
__device__ void task_temp_add(const DevEnv &e, const Lds &L, double *lds, const Task &tk) {
  const int tu = tk.i[0], tv = tk.i[1], tp = tk.i[2], rp = tk.i[3], bu = tk.i[4], bv = tk.i[5];
  const int tT = tk.i[6], rT = tk.i[7];
  const int k1 = e.bcols[tu], k2 = e.bcols[bu];
  const int kk = k1 + k2;
  if (kk == 0) return;
  const int mt = e.size[tT], mr = e.size[rT];
  const int qa = mt < kk ? mt : kk, qb = mr < kk ? mr : kk;
  // capacity check against the allocations below (work areas of waves 0 and 1)
  {
    const long need0 = (long)(mt | 1) * kk + (kk | 1) + (long)(qa | 1) * qb + (long)(qb | 1) * qb +
                       (long)(qa | 1) * qa + (long)(mt | 1) * (qa > qb ? qa : qb) + 3L * (kk | 1) * (kk + 1);
    const long need1 = (long)(mr | 1) * kk + (kk | 1) + (long)(mr | 1) * (qa > qb ? qa : qb);
    if (need0 > TEMP_WAVE_MAX || need1 > TEMP_WAVE_MAX) { task_temp_add_wg(e, L, tk); return; }
  }
  const int w = wave_id(), lane = lane_id();
  // only waves 0 and 1 hold matrices here: each gets the LDS of half of the
  // waves (the small vectors of the last wave hold the ranking)
  const Wv W0 = wave_areas_of(lds, e, NWAVE - 1);
  constexpr int HALF = (NWAVE / 2) * (WREG + WSMALL) - WSMALL;
  WvAlloc a0 = WvAlloc{lds, e.wscr, e.err, 0, 0, HALF};
  WvAlloc a1 = WvAlloc{lds + (NWAVE / 2) * (WREG + WSMALL), e.wscr + WGLOB, e.err, 0, 0, HALF};
  const MV X0 = a0.take(mt, kk), X1 = a1.take(mr, kk);
  double *tau0 = a0.take(kk, 1).p, *tau1 = a1.take(kk, 1).p;
  if (w < 2) {
    const int rows = w == 0 ? mt : mr;
    const MV X = w == 0 ? X0 : X1;
    const MV T = w == 0 ? bufrows(e, tu, tT) : bufrows(e, tv, rT);
    const int cl = w == 0 ? tp : rp, clT = w == 0 ? tT : rT;
    const int at = e.offset[cl] - e.offset[clT], nt = e.size[cl];
    const MV U = bufrows(e, w == 0 ? bu : bv, cl);
    for (int q = lane; q < rows * kk; q += 64) {
      const int i = q % rows, j = q / rows;
      X(i, j) = j < k1 ? T(i, j) : ((i >= at && i < at + nt) ? U(i - at, j - k1) : 0.0);
    }
    wave_sync();
    wv_qr(rows, kk, X, w == 0 ? tau0 : tau1);
  }
  __syncthreads();
  // core C = Ra Rb^* (qa x qb) and its SVD on wave 0.  G = C, or C^* when C
  // is wide (grow >= nj).  Above PRECOND_MIN columns the SVD is
  // QR-preconditioned: G = Qg R, R^* = Q2 R2, one-sided Jacobi on
  // X = R2^* with the rotations J accumulated, so that
  // G = (Qg X J) (Q2 J)^* with the columns of X J orthogonal.
  const bool tr = qa < qb;
  const int nj = tr ? qa : qb;        // columns rotated
  const int grow = tr ? qb : qa;
  const bool pre = nj > PRECOND_MIN;
  const MV C = a0.take(qa, qb), J = a0.take(nj, nj);
  const MV G = tr ? mv_t(C) : C;      // grow x nj
  double *taug = a0.take(nj, 1).p, *tauy = a0.take(nj, 1).p;
  const MV Y = a0.take(nj, nj), X = a0.take(nj, nj);
  const MV Gs = pre ? X : G;          // the matrix whose columns are rotated
  if (w == 0) {
    for (int q = lane; q < qa * qb; q += 64) {
      const int i = q % qa, j = q / qa;
      double acc = 0.0;
      for (int l = (i > j ? i : j); l < kk; ++l) acc = fma(X0(i, l), X1(j, l), acc);
      C(i, j) = acc;
    }
    for (int q = lane; q < nj * nj; q += 64) J(q % nj, q / nj) = (q % nj == q / nj) ? 1.0 : 0.0;
    wave_sync();
    if (pre) {
      wv_qr(grow, nj, G, taug);
      for (int q = lane; q < nj * nj; q += 64) {
        const int i = q % nj, j = q / nj;
        Y(i, j) = i >= j ? G(j, i) : 0.0;
      }
      wave_sync();
      wv_qr(nj, nj, Y, tauy);
      for (int q = lane; q < nj * nj; q += 64) {
        const int i = q % nj, j = q / nj;
        X(i, j) = i >= j ? Y(j, i) : 0.0;
      }
      wave_sync();
    }
    const int srow = pre ? nj : grow;
    MV Jv = J;
    wave_jacobi(srow, nj, Gs, &Jv);
    wv_colnorms_sorted(srow, nj, Gs, W0.sig, W0.ord);
    if (lane == 0) {
      double tau = 0.0;
      if (e.mode == 0) {
        double s2 = 0.0;
        for (int j = 0; j < nj; ++j) s2 += W0.sig[j] * W0.sig[j];
        tau = e.eps * sqrt(s2);
      } else if (e.mode == 1) {
        tau = e.eps * (nj > 0 ? W0.sig[W0.ord[0]] : 0.0);
      }
      int r = 0;
      for (int j = 0; j < nj; ++j) r += W0.sig[W0.ord[j]] > tau ? 1 : 0;
      W0.ord[127] = r;
    }
    count(e, fl_qr(mt, kk) + fl_qr(mr, kk) + fl_gemm(qa, qb, kk) + fl_svd(qa, qb) +
             14.0 * (double)nj * nj * nj);
  }
  __syncthreads();
  const int r = W0.ord[127];
  if (r > e.rank_cap) { set_error(e, E_RANK_CAP, tT); return; }
  // TU = Qa (U Sigma)_r on wave 0, TV = Qb W_r on wave 1.  With G = C,
  // U Sigma = (Qg) Gs J-rotated columns and W = (Q2) J; with G = C^* the two
  // roles are exchanged.  (Qg, Q2 only when preconditioned.)
  if (w < 2) {
    const int rows = w == 0 ? mt : mr;
    const int qx = pre ? nj : (w == 0 ? qa : qb);
    WvAlloc az = w == 0 ? a0 : a1;
    const MV Z = az.take(rows, r > 0 ? r : 1);
    const bool rotated = (w == 0) != tr;   // this side takes the rotated columns
    for (int q = lane; q < rows * r; q += 64) {
      const int i = q % rows, j = q / rows;
      const int c = W0.ord[j];
      double v = 0.0;
      if (i < qx) {
        if (rotated) v = w == 0 ? Gs(i, c) : (W0.sig[c] > 0.0 ? Gs(i, c) / W0.sig[c] : 0.0);
        else v = w == 0 ? J(i, c) * W0.sig[c] : J(i, c);
      }
      Z(i, j) = v;
    }
    wave_sync();
    if (pre) {
      if (rotated) wv_apply_q(grow, nj, G, taug, Z, r);   // Qg
      else wv_apply_q(nj, nj, Y, tauy, Z, r);             // Q2
    }
    wv_apply_q(rows, kk, w == 0 ? X0 : X1, w == 0 ? tau0 : tau1, Z, r);
    const MV out = w == 0 ? bufrows(e, tu, tT) : bufrows(e, tv, rT);
    for (int q = lane; q < rows * r; q += 64) out(q % rows, q / rows) = Z(q % rows, q / rows);
    if (lane == 0 && e.flops) e.flops[1 + w] += 4.0 * rows * kk * r;
  }
  if (threadIdx.x == 0) { e.bcols[tu] = r; e.bcols[tv] = r; }
  __syncthreads();
}

__device__ void task_potrf(const DevEnv &e, const Lds &L, int bcc, int t) {
  const int info = wg_potrf(e.size[t], Nslot(e, bcc), L.iw);
  count(e, (double)e.size[t] * e.size[t] * e.size[t] / 3.0);
  if (info) set_error(e, E_NOT_SPD, t);
}

// LR factorisation of a diagonal leaf without pivoting (leaf case of the
// LR recursion of Section 3): N_cc <- (L - I) + R.
__device__ void task_getrf(const DevEnv &e, const Lds &L, int bcc, int t) {
  const int n = e.size[t];
  const int info = wg_getrf_nopiv(n, Nslot(e, bcc), L.iw);
  count(e, 2.0 * n * n * n / 3.0);
  if (info) set_error(e, E_ZERO_PIVOT, t);
}

// Solve with a diagonal leaf on an inadmissible leaf b in place:
// TRI_CHOL  b = (r, c): N_b <- N_b L_cc^{-T}  (Cholesky factor);
// TRI_L_UNIT b = (c, r): N_b <- L_cc^{-1} N_b (unit lower LR factor);
// TRI_R_ADJ b = (r, c): N_b <- N_b R_cc^{-1}  (upper LR factor), as
//                        N_b^T <- R_cc^{-T} N_b^T.
__device__ void task_trsm(const DevEnv &e, int b, int bcc, int kind) {
  const int c = e.brow[bcc];
  const int nc = e.size[c];
  if (kind == TRI_CHOL) {
    const int r = e.brow[b];
    wg_trsm_right_lt(e.size[r], nc, Nslot(e, bcc), Nslot(e, b));
    count(e, (double)e.size[r] * nc * nc);
  } else if (kind == TRI_L_UNIT) {
    const int m = e.size[e.bcol[b]];
    wg_trsv_ex(nc, m, Nslot(e, bcc), Nslot(e, b), 0, true, true);
    count(e, (double)m * nc * nc);
  } else {
    const int m = e.size[e.brow[b]];
    wg_trsv_ex(nc, m, Nslot(e, bcc), mv_t(Nslot(e, b)), 1, true, false);
    count(e, (double)m * nc * nc);
  }
}

// buf|_c <- T^{-1} buf|_c with the triangle of the diagonal leaf named by
// kind (TRI_CHOL: L^{-1}, or L^{-T} if trans).
__device__ void task_trsv(const DevEnv &e, int bcc, int bi, int trans, int kind) {
  if (e.bcols[bi] == 0) return;   // no columns
  const int c = e.brow[bcc];
  if (kind == TRI_CHOL) wg_trsv_lower(e.size[c], e.bcols[bi], Nslot(e, bcc), bufrows(e, bi, c), trans);
  else if (kind == TRI_L_UNIT) wg_trsv_ex(e.size[c], e.bcols[bi], Nslot(e, bcc), bufrows(e, bi, c), 0, true, true);
  else if (kind == TRI_R_ADJ) wg_trsv_ex(e.size[c], e.bcols[bi], Nslot(e, bcc), bufrows(e, bi, c), 1, true, false);
  else wg_trsv_ex(e.size[c], e.bcols[bi], Nslot(e, bcc), bufrows(e, bi, c), 0, false, false);
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

// Inverse of the lower triangular diagonal leaf (c, c) in place (leaf case
// of the triangular inversion).
__device__ void task_trtri(const DevEnv &e, int bcc) {
  const int n = e.size[e.brow[bcc]];
  wg_trtri_lower(n, Nslot(e, bcc));
  count(e, (double)n * n * n / 3.0);
}

// buf|_c <- tril(N_cc) buf|_c (trans: transposed), the leaf case of the
// product with a lower triangular matrix.
__device__ void task_trmv(const DevEnv &e, int bcc, int bi, int trans) {
  if (e.bcols[bi] == 0) return;   // no columns
  const int c = e.brow[bcc];
  wg_trmv_lower(e.size[c], e.bcols[bi], Nslot(e, bcc), bufrows(e, bi, c), trans);
  count(e, (double)e.size[c] * e.size[c] * e.bcols[bi]);
}

// Product of an inadmissible leaf with a lower triangular diagonal leaf, in
// place: N_b <- tril(N_cc) N_b (side 0, b = (c, r)) or N_b <- N_b tril(N_cc)
// (side 1, b = (r, c)), the second as N_b^T <- tril(N_cc)^T N_b^T.
__device__ void task_near_trmul(const DevEnv &e, int b, int bcc, int side) {
  const int nc = e.size[e.brow[bcc]];
  MV N = Nslot(e, b);
  if (side == 0) wg_trmv_lower(nc, e.size[e.bcol[b]], Nslot(e, bcc), N, 0);
  else wg_trmv_lower(nc, e.size[e.brow[b]], Nslot(e, bcc), mv_t(N), 1);
  count(e, (double)nc * nc * (side == 0 ? e.size[e.bcol[b]] : e.size[e.brow[b]]));
}

// Negate every stored leaf block listed in aux[off .. off + cnt): the
// coupling matrix of an admissible leaf, the dense block of an
// inadmissible one.  One wave per block.
__device__ void task_neg(const DevEnv &e, const int *aux, int off, int cnt) {
  const int lane = lane_id();
  for (int q = wave_id(); q < cnt; q += num_waves()) {
    const int b = aux[off + q];
    if (e.bkind[b] == 1) {
      MV S = Sslot(e, b);
      const int kt = e.k[0][e.brow[b]], ks = e.k[1][e.bcol[b]];
      for (int p = lane; p < kt * ks; p += 64) S(p % kt, p / kt) = -S(p % kt, p / kt);
    } else {
      MV N = Nslot(e, b);
      const int mt = e.size[e.brow[b]], ms = e.size[e.bcol[b]];
      for (int p = lane; p < mt * ms; p += 64) N(p % mt, p / mt) = -N(p % mt, p / mt);
    }
  }
  __syncthreads();
}

// ============================================================ interpreter
// One workgroup replays one task list against one matrix.
__device__ __forceinline__ void interp_run(const Task *__restrict__ tasks, int ntask,
                                           const DevEnv *__restrict__ env, const int *__restrict__ aux) {
  extern __shared__ double lds_raw[];
  const DevEnv &e0 = *env;
  const Lds L = lds_layout(lds_raw);
  if (e0.err[0] != 0) return;
  Task nxt = ntask > 0 ? tasks[0] : Task{};
  for (int it = 0; it < ntask; ++it) {
    __syncthreads();
    const Task tk = nxt;
    if (it + 1 < ntask) nxt = tasks[it + 1];   // fetched while this task runs
    // the matrix whose data the task reads; every environment of one list
    // shares the target's work areas, error flag and counters
    const DevEnv &e = env[tk.env];
    const unsigned long long t0 = e.prof ? wall_clock64() : 0ull;
    switch (tk.op) {
      case OP_ADDLR:
      case OP_ADDLR_ACC: task_addlr_tk(e, L, lds_raw, tk); break;
      case OP_EXPAND: task_expand(e, tk.i[0], tk.i[1], tk.i[2]); break;
      case OP_BAPPLY: {
        task_bapply(e, L, tk.i[0], tk.i[1], tk.i[2], tk.i[3], tk.alpha, tk.beta);
        if (e.prof && threadIdx.x == 0) {
          // size class by the number of clusters below the destination cluster
          const int dr = tk.i[1] ? e.bcol[tk.i[0]] : e.brow[tk.i[0]];
          int nclu = 0;
          for (int lv = e.level[dr]; lv < e.nlev; ++lv) nclu += dhi(e, dr, lv) - dlo(e, dr, lv);
          const int cls = nclu <= 1 ? 0 : nclu <= 3 ? 1 : nclu <= 15 ? 2 : nclu <= 63 ? 3 : nclu <= 255 ? 4 : 5;
          e.prof[PROF_BAPPLY + cls] += wall_clock64() - t0;
          e.prof[PROF_BAPPLY + 8 + cls] += 1;
        }
        break;
      }
      case OP_RMUL_S: task_rmul_s(e, tk.i[0], tk.i[1], tk.i[2], tk.i[3], tk.i[4], tk.alpha); break;
      case OP_COPY_NEAR: task_copy_near(e, tk.i[0], tk.i[1], tk.i[2], tk.alpha); break;
      case OP_IDENT: task_ident(e, tk.i[0], tk.i[1], tk.i[2], tk.i[3]); break;
      case OP_NEAR_ADD: task_near_add(e, tk.i[0], tk.i[1], tk.i[2], tk.alpha); break;
      case OP_TEMP_INIT: task_temp_init(e, tk.i[0], tk.i[1], tk.i[2], tk.i[3]); break;
      case OP_TEMP_ADD: {
        task_temp_add(e, L, lds_raw, tk);
        if (e.prof && threadIdx.x == 0) {
          const int rows = e.size[tk.i[6]] > e.size[tk.i[7]] ? e.size[tk.i[6]] : e.size[tk.i[7]];
          const int cls = rows <= 32 ? 0 : rows <= 128 ? 1 : rows <= 512 ? 2 : rows <= 2048 ? 3 : 4;
          e.prof[PROF_TEMP + cls] += wall_clock64() - t0;
          e.prof[PROF_TEMP + 8 + cls] += 1;
        }
        break;
      }
      case OP_POTRF: task_potrf(e, L, tk.i[0], tk.i[1]); break;
      case OP_TRSM: task_trsm(e, tk.i[0], tk.i[1], tk.i[2]); break;
      case OP_TRSV: task_trsv(e, tk.i[0], tk.i[1], tk.i[2], tk.i[3]); break;
      case OP_GETRF: task_getrf(e, L, tk.i[0], tk.i[1]); break;
      case OP_SUB: task_sub(e, tk.i[0], tk.i[1], tk.i[2], tk.i[3]); break;
      case OP_COPY: task_copy(e, tk.i[0], tk.i[1], tk.i[2]); break;
      case OP_SV_ZERO: task_sv_zero(e, tk.i[0], tk.i[1], tk.i[2]); break;
      case OP_SV_PUSH: task_sv_push(e, tk.i[0], tk.i[1], tk.i[2]); break;
      case OP_SV_LEAF: task_sv_leaf(e, tk.i[0], tk.i[1], tk.i[2]); break;
      case OP_SV_CROSS: task_sv_cross(e, aux, tk.i[0], tk.i[1], tk.i[2], tk.i[3]); break;
      case OP_SV_UP: task_sv_up(e, tk.i[0], tk.i[1], tk.i[2]); break;
      case OP_TRTRI: task_trtri(e, tk.i[0]); break;
      case OP_TRMV: task_trmv(e, tk.i[0], tk.i[1], tk.i[2]); break;
      case OP_NEG: task_neg(e, aux, tk.i[0], tk.i[1]); break;
      case OP_NEAR_TRMUL: task_near_trmul(e, tk.i[0], tk.i[1], tk.i[2]); break;
      default: set_error(e, E_ARG, tk.op); break;
    }
    if (e.prof && threadIdx.x == 0 && tk.op > 0 && tk.op < 32) {
      e.prof[PROF_COUNT + tk.op] += 1;
      e.prof[PROF_TICKS + tk.op] += wall_clock64() - t0;
    }
    // only these kinds can record an error (set_error ends with a barrier)
    if (tk.op == OP_ADDLR || tk.op == OP_ADDLR_ACC || tk.op == OP_POTRF || tk.op == OP_GETRF ||
        tk.op == OP_TEMP_ADD || tk.op <= 0 ||
        tk.op >= 32) {
      __syncthreads();
      if (e0.err[0] != 0) return;
    }
  }
}

__global__ __launch_bounds__(NT) void k_interp(const Task *__restrict__ tasks, int ntask,
                                               const DevEnv *__restrict__ env, const int *__restrict__ aux) {
  interp_run(tasks, ntask, env, aux);
}

// Independent matrices in one launch: workgroup i replays items[i] (its own
// task list, matrix and work areas; nothing is shared between workgroups).
__global__ __launch_bounds__(NT) void k_interp_batch(const BatchItem *__restrict__ items) {
  const BatchItem it = items[blockIdx.x];
  if (it.gate != nullptr && *it.gate == 0) return;
  interp_run(it.tasks, it.ntask, it.env, it.aux);
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

__global__ void k_fill_double(double *p, int n, double v) {
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

// ------------------------------------------- batched PCG, all columns per launch
// The graph form of the batched PCG: one launch per operation for all
// right-hand sides (blockIdx.y = column), each gated by the column's active
// flag.  Per column the arithmetic is that of the single-column kernels
// above (same row loops, same partial-sum blocking of the dot products), so
// both forms give the same numbers.
enum : int { PCG_DOT_PQ = 0, PCG_DOT_RR = 1, PCG_DOT_RZ = 2 };

__global__ void k_bpcg_spmv(const PcgCol *__restrict__ cols, const int *__restrict__ act) {
  const int c = blockIdx.y;
  if (act[c] == 0) return;
  const PcgCol k = cols[c];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k.n; i += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t p = k.rp[i]; p < k.rp[i + 1]; ++p) s = fma(k.v[p], k.p[k.ci[p]], s);
    k.q[i] = s;
  }
}

__global__ void k_bpcg_dot_partial(const PcgCol *__restrict__ cols, const int *__restrict__ act, int which) {
  const int c = blockIdx.y;
  if (act[c] == 0) return;
  const PcgCol k = cols[c];
  const double *a = which == PCG_DOT_PQ ? k.p : k.r;
  const double *b = which == PCG_DOT_PQ ? k.q : (which == PCG_DOT_RR ? k.r : k.z);
  __shared__ double red[16];
  double s = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k.n; i += gridDim.x * blockDim.x) s = fma(a[i], b[i], s);
  s = wave_sum(s);
  if (lane_id() == 0) red[wave_id()] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < num_waves(); ++w) t += red[w];
    k.part[blockIdx.x] = t;
  }
}

__global__ void k_bpcg_dot_final(const PcgCol *__restrict__ cols, const int *__restrict__ act, int np, int slot) {
  const int c = blockIdx.x;
  if (act[c] == 0) return;
  const PcgCol k = cols[c];
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += k.part[i];
  s = wave_sum(s);
  if (lane_id() == 0) red[wave_id()] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < num_waves(); ++w) t += red[w];
    k.sc[slot] = t;
  }
}

__global__ void k_bpcg_update_xr(const PcgCol *__restrict__ cols, const int *__restrict__ act) {
  const int c = blockIdx.y;
  if (act[c] == 0) return;
  const PcgCol k = cols[c];
  const double alpha = k.sc[0] / k.sc[1];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k.n; i += gridDim.x * blockDim.x) {
    k.x[i] = fma(alpha, k.p[i], k.x[i]);
    k.r[i] = fma(-alpha, k.q[i], k.r[i]);
  }
}

__global__ void k_bpcg_update_p(const PcgCol *__restrict__ cols, const int *__restrict__ act) {
  const int c = blockIdx.y;
  if (act[c] == 0) return;
  const PcgCol k = cols[c];
  const double beta = k.sc[2] / k.sc[0];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k.n; i += gridDim.x * blockDim.x)
    k.p[i] = fma(beta, k.p[i], k.z[i]);
}

__global__ void k_bpcg_next(const PcgCol *__restrict__ cols, const int *__restrict__ act, int ncol) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncol; c += gridDim.x * blockDim.x)
    if (act[c] != 0) cols[c].sc[0] = cols[c].sc[2];
}

// Convergence test after x and r are updated (one workgroup): a column that
// ran this iteration counts it, stores ||r|| / ||b|| and stops when that is
// at most rtol (converged) or the iteration limit is reached; a system stays
// active while one of its columns is.
__global__ void k_bpcg_check(const PcgCol *__restrict__ cols, PcgCtl ctl, int ncol, int nsys, double rtol,
                             int maxit) {
  for (int y = threadIdx.x; y < nsys; y += blockDim.x) ctl.sys_act[y] = 0;
  __syncthreads();
  int cnt = 0;
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
    if (ctl.act[c] == 0) continue;
    const int it = ctl.it[c] + 1;
    ctl.it[c] = it;
    const double rel = sqrt(cols[c].sc[3]) / cols[c].nb;
    ctl.rel[c] = rel;
    int a = 1;
    if (rel <= rtol) { ctl.conv[c] = 1; a = 0; }
    else if (it >= maxit) a = 0;
    ctl.act[c] = a;
    if (a) { ctl.sys_act[cols[c].sys] = 1; ++cnt; }
  }
  __shared__ int red[16];
  int s = cnt;
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane_id() == 0) red[wave_id()] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < num_waves(); ++w) t += red[w];
    *ctl.nact = t;
  }
}

}  // namespace h2
