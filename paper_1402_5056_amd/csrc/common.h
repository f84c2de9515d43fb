// Shared definitions of the h2lr host code and device kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace h2 {

constexpr int KC = 32;     // rank capacity of basis / coupling slots
constexpr int KM = 64;     // capacity of an extended rank k + k'
constexpr int LS = 32;     // leaf capacity (rows of a leaf basis, nearfield side)
constexpr int BC = 64;     // columns of a work buffer (row-major, ld = BC)
constexpr int NT = 512;    // threads of the task interpreter workgroup
constexpr int KPMAX = KM - KC;  // largest update rank k'

// Device error codes written to err[0] (mirrors h2_status).
enum : int { E_OK = 0, E_NOT_SPD = -4, E_RANK_CAP = -5, E_ARG = -1, E_ZERO_PIVOT = -9, E_SCRATCH = -100 };

// Work buffers: n x BC row-major arrays indexed by cluster-order rows.
enum Buf : int {
  B_U, B_V, B_A, B_B, B_W, B_WP, B_I, B_X, B_Y,
  B_T0U, B_T0V, B_T1U, B_T1V, B_T2U, B_T2V, B_T3U, B_T3V,
  NBUF
};

enum Op : int {
  OP_ADDLR = 1,      // i0 block, i1 bufX, i2 bufY
  OP_EXPAND,         // i0 side, i1 cluster, i2 buf       -> buf rows = expanded basis, cols = k
  OP_BAPPLY,         // i0 block, i1 trans, i2 in, i3 out; alpha, beta
  OP_RMUL_S,         // i0 in, i1 out, i2 block, i3 transS, i4 rows cluster; alpha
  OP_COPY_NEAR,      // i0 block, i1 out, i2 trans; alpha -> rows of row (trans: column) cluster
  OP_IDENT,          // i0 cluster, i1 buf, i2 first col, i3 ncols
  OP_NEAR_ADD,       // i0 block, i1 U, i2 V; alpha
  OP_TEMP_INIT,      // i0 U, i1 V, i2 row cluster, i3 col cluster
  OP_TEMP_ADD,       // i0 tU, i1 tV, i2 t', i3 r', i4 U, i5 V, i6 temp row cluster, i7 temp col cluster
  OP_POTRF,          // i0 leaf cluster
  OP_TRSM,           // i0 near block, i1 diagonal leaf block, i2 kind (TRI_*)
  OP_TRSV,           // i0 diagonal leaf block, i1 buf, i2 trans (kind TRI_CHOL), i3 kind (TRI_*)
  OP_SUB,            // i0 A, i1 B, i2 out, i3 cluster
  OP_COPY,           // i0 A, i1 out, i2 cluster
  OP_SV_ZERO,        // i0 cluster, i1 buf, i2 trans   substitution: clear the coupling sums of the subtree
  OP_SV_PUSH,        // i0 cluster, i1 buf, i2 trans   substitution: coupling sums to the sons
  OP_SV_LEAF,        // i0 diagonal leaf block, i1 buf, i2 trans
  OP_SV_CROSS,       // i0 aux offset, i1 groups, i2 buf, i3 trans  leaves of (c2, c1), solved -> unsolved part
  OP_SV_UP,          // i0 cluster, i1 buf, i2 trans   forward transformation of a solved cluster
  OP_TRTRI,          // i0 diagonal leaf block         N <- inverse of its lower triangle
  OP_TRMV,           // i0 diagonal leaf block, i1 buf, i2 trans   buf rows <- tril(N) (or its transpose) buf rows
  OP_NEG,            // i0 aux offset, i1 count        negate the stored leaf blocks listed in aux
  OP_NEAR_TRMUL,     // i0 near block, i1 diagonal leaf block, i2 side   N <- tril(N_cc) N (0) or N tril(N_cc) (1)
  OP_GETRF,          // i0 diagonal leaf block, i1 cluster   LR of the leaf without pivoting
  OP_ADDLR_ACC,      // i0 block, i1 temporaries (pairs T0..T3)  add them: one update each, or accumulated
};

// Which triangle of a diagonal leaf a solve uses.  TRI_CHOL: the Cholesky
// factor L (lower; trsv: L^{-1} or L^{-T} by trans, trsm: N <- N L^{-T});
// the LR factor of a leaf holds unit lower L and upper R:
// TRI_L_UNIT: L^{-1} x (trsm: N <- L^{-1} N); TRI_R_ADJ: R^{-T} x (trsm:
// N <- N R^{-1}); TRI_R: R^{-1} x.
enum : int { TRI_CHOL = 0, TRI_L_UNIT = 1, TRI_R_ADJ = 2, TRI_R = 3 };

struct Task {
  int op;
  int i[8];
  int env;   // index of the environment whose matrix data the task reads (0: the target)
  double alpha, beta;
};

// Everything a device task needs, passed by value to the interpreter.
struct DevEnv {
  int n, nc, depth, nlev;          // nlev = depth + 1
  int rank_cap, mode;              // truncation
  double eps;
  int prec;                        // 0: FP64 products; 1: coupling/transfer products in FP32
  int acc;                         // 1: accumulate the temporaries of a product target
  double lvq;                      // level factor q of the recompression threshold (1: none)
  // cluster tree
  const int *offset, *size, *son0, *son1, *parent, *level;
  const int *desc_lo, *desc_hi;    // nc x nlev: descendants of t at level l = [lo, hi)
  // block tree
  const int *brow, *bcol, *bkind, *bfirst, *bnsons;
  const int *bslot;                // stored slot of a leaf block, -1 otherwise
  const int *rowptr, *rowidx;      // row(t): stored admissible blocks, by block id
  const int *colptr, *colidx;      // col(s)
  const int *nrowptr, *nrowidx;    // stored inadmissible leaves by row cluster
  const int *ncolptr, *ncolidx;    // ... by column cluster
  // matrix data: index 0 row basis V, 1 column basis W
  int *k[2];
  double *leaf[2];                 // nc slots LS x KC, col-major ld LS
  double *E[2];                    // nc slots KC x KC, ld KC (k_t x k_father)
  double *rho[2];                  // nc slots KC x KC
  int *rho_m[2];                   // rows of rho
  double *S;                       // adm slots KC x KC (k_t x k_s)
  double *N;                       // near slots LS x LS (#t x #s)
  // update workspace (per cluster)
  double *wrho[2]; int *wrho_m[2];
  double *wB[2]; int *wB_m[2];
  double *wR[2]; int *wnewk[2];
  // products with sub-blocks
  double *xh, *yh;                 // nc slots KC x BC row-major
  // work buffers
  double *buf[NBUF];
  int *bcols;
  int *err;                        // err[0] code, err[1] info
  unsigned long long *prof;        // optional: per-op counts/ticks, update stage ticks
  double *flops;                   // algorithmic flops: [0] workgroup code, [1 + w] wave w
  double *wscr;                    // per-wave global overflow work areas
};

// One entry of a batched interpreter launch.
struct BatchItem {
  const Task *tasks;
  const DevEnv *env;
  const int *aux;
  int ntask;
  int pad;
  const int *gate;   // optional: the workgroup skips its list while *gate == 0
};

// One right-hand side of the batched PCG in its graph form: the system's
// CSR matrix, the column's vectors (length n), its dot-product partial sums
// and scalars (sc[0] = r.z, sc[1] = p.q, sc[2] = new r.z, sc[3] = r.r),
// ||b|| and the index of its system.
struct PcgCol {
  const int64_t *rp;
  const int *ci;
  const double *v;
  double *x, *r, *z, *p, *q, *part, *sc;
  double nb;
  int n, sys;
};

// Device state of the batched PCG graph form, per column: active flag,
// iterations, converged flag, relative residual; per system: any column
// active; and the number of active columns.
struct PcgCtl {
  int *act, *it, *conv, *sys_act, *nact;
  double *rel;
};

// Layout of the optional profile counters (ticks of the 100 MHz wall clock).
constexpr int PROF_COUNT = 0;      // [0, 32): tasks executed per op
constexpr int PROF_TICKS = 32;     // [32, 64): ticks per op
constexpr int PROF_STAGE = 64;     // [64, 80): ticks per update stage
constexpr int PROF_BAPPLY = 80;   // [80, 88): ticks of sub-block products by size class, [88, 96): counts
constexpr int PROF_WAVE = 96;     // [96, 128): per-wave ticks / counts inside update stages
constexpr int PROF_LEVEL = 128;    // [128, 144): ticks of low-rank updates by level of t0, [144, 160): counts
constexpr int PROF_LEAFSTAGE = 160; // [160, 168): ticks per update stage, updates of leaf blocks only
constexpr int PROF_TEMP = 176;     // [176, 184): ticks of truncated additions by row count class, [184, 192): counts
constexpr int PROF_SFLOPS = 192;   // [192, 198): algorithmic flops of the update steps a4..a9
constexpr int PROF_SBYTES = 198;   // [198, 204): algorithmic bytes of the update steps a4..a9
constexpr int PROF_LEN = 204;
// update steps (a4 R-factors, a5 weights, a6 recompression, a7 couplings,
// a8 R-factor path refresh and transfer update, a9 nearfield)
enum : int { ST_A4 = 0, ST_A5, ST_A6, ST_A7, ST_A8, ST_A9 };

}  // namespace h2
