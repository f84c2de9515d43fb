// Host side of the h2lr C ABI: trees, H^2 storage in flat device arrays,
// the planner that turns the recursive algorithms into task lists, and the
// launches of the task interpreter and helper kernels.
#include "tasks.hip"
#include "h2lr.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

using namespace h2;

namespace {

thread_local std::string g_last_error;

struct H2Error : std::runtime_error {
  h2_status code;
  H2Error(h2_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess)                                                            \
      throw H2Error(e_ == hipErrorOutOfMemory ? H2_ERR_NOMEM : H2_ERR_HIP,           \
                    std::string(#x) + ": " + hipGetErrorString(e_));                 \
  } while (0)

#define REQUIRE(cond, msg) \
  do { if (!(cond)) throw H2Error(H2_ERR_ARG, msg); } while (0)

template <class F>
h2_status guarded(F &&f) {
  try {
    f();
    return H2_OK;
  } catch (const H2Error &e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return H2_ERR_NOMEM;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return H2_ERR_HIP;
  }
}

// The device's default memory pool keeps freed memory for reuse instead of
// returning it to the system (set once per device before its first
// stream-ordered allocation).
static void keep_pool_memory(hipStream_t s) {
  static std::mutex mu;
  static std::vector<int> done;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  (void)s;
  std::lock_guard<std::mutex> lock(mu);
  if (std::find(done.begin(), done.end(), dev) != done.end()) return;
  hipMemPool_t pool;
  HIPCHK(hipDeviceGetDefaultMemPool(&pool, dev));
  uint64_t keep = ~0ull;
  HIPCHK(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
  done.push_back(dev);
}

// Owning device allocation.  alloc(): hipMalloc / hipFree.  alloc_on(n, s):
// stream-ordered (hipMallocAsync on s, complete when the call returns;
// hipFreeAsync on s when released), so that freeing a matrix does not wait
// for the work of other streams on the device.
template <class T>
struct Dev {
  T *p = nullptr;
  size_t n = 0;
  hipStream_t s = nullptr;
  bool ordered = false;
  Dev() = default;
  Dev(const Dev &) = delete;
  Dev &operator=(const Dev &) = delete;
  ~Dev() { release(); }
  void release() {
    if (p) {
      if (ordered) (void)hipFreeAsync(p, s);
      else (void)hipFree(p);
      p = nullptr;
    }
  }
  void alloc(size_t count) {
    release();
    n = count;
    ordered = false;
    if (count) HIPCHK(hipMalloc(&p, count * sizeof(T)));
  }
  void alloc_on(size_t count, hipStream_t st) {
    release();
    n = count;
    s = st;
    ordered = true;
    if (count) {
      keep_pool_memory(st);
      HIPCHK(hipMallocAsync(reinterpret_cast<void **>(&p), count * sizeof(T), st));
      HIPCHK(hipStreamSynchronize(st));
    }
  }
  void upload(const std::vector<T> &h, hipStream_t st) {
    alloc_on(h.size(), st);
    if (n) HIPCHK(hipMemcpyAsync(p, h.data(), n * sizeof(T), hipMemcpyHostToDevice, st));
  }
  void zero(hipStream_t st) { if (n) HIPCHK(hipMemsetAsync(p, 0, n * sizeof(T), st)); }
};

}  // namespace

// ====================================================================== ctx
struct h2_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
};

// ============================================================= cluster tree
struct h2_ctree_s {
  h2_ctx ctx;
  int64_t n = 0;
  int dim = 0, leaf = 0, nc = 0, depth = 0, nlev = 0;
  std::vector<int64_t> perm;
  std::vector<int> offset, size, level, son0, son1, parent;
  std::vector<char> uni;         // 1: the sons are two domains separated by an interface
  std::vector<int64_t> lo, hi;   // nc x dim
  std::vector<int> desc_lo, desc_hi;
  Dev<int64_t> d_perm;
  Dev<int> d_offset, d_size, d_level, d_son0, d_son1, d_parent, d_desc_lo, d_desc_hi;
};

// Roles of the clusters of a domain-decomposition tree: a domain is cut by an
// interface hyperplane, a union holds the two domains of one cut, every other
// cluster (interfaces and their descendants) is bisected.
enum { ROLE_DOMAIN = 0, ROLE_UNION = 1, ROLE_OTHER = 2 };

static void build_ctree(h2_ctree_s &ct, const int32_t *coords, bool dd) {
  const int64_t n = ct.n;
  const int dim = ct.dim;
  ct.perm.resize(n);
  for (int64_t i = 0; i < n; ++i) ct.perm[i] = i;
  std::vector<char> role;
  std::vector<int> cut;
  std::deque<int> q;
  auto add = [&](int off, int sz, int lev, int par, char rl, int ct_cut) {
    const int id = (int)ct.offset.size();
    ct.offset.push_back(off); ct.size.push_back(sz); ct.level.push_back(lev);
    ct.son0.push_back(-1); ct.son1.push_back(-1); ct.parent.push_back(par);
    role.push_back(rl); cut.push_back(ct_cut);
    for (int d = 0; d < dim; ++d) {
      int64_t a = INT64_MAX, b = INT64_MIN;
      for (int i = off; i < off + sz; ++i) {
        const int64_t v = coords[ct.perm[i] * dim + d];
        a = std::min(a, v); b = std::max(b, v);
      }
      ct.lo.push_back(a); ct.hi.push_back(b);
    }
    q.push_back(id);
    return id;
  };
  add(0, (int)n, 0, -1, dd ? ROLE_DOMAIN : ROLE_OTHER, 0);
  std::vector<int64_t> tmp;
  while (!q.empty()) {
    const int t = q.front();
    q.pop_front();
    const int off = ct.offset[t], sz = ct.size[t];
    if (sz <= ct.leaf) continue;
    if (role[t] == ROLE_UNION) {
      // the father already placed the first domain before the second
      const int s0 = add(off, cut[t], ct.level[t] + 1, t, ROLE_DOMAIN, 0);
      const int s1 = add(off + cut[t], sz - cut[t], ct.level[t] + 1, t, ROLE_DOMAIN, 0);
      ct.son0[t] = s0; ct.son1[t] = s1;
      continue;
    }
    int dsplit = 0;
    int64_t best = -1;
    for (int d = 0; d < dim; ++d) {
      const int64_t ext = ct.hi[t * dim + d] - ct.lo[t * dim + d];
      if (ext > best) { best = ext; dsplit = d; }
    }
    const int64_t mid2 = ct.lo[t * dim + dsplit] + ct.hi[t * dim + dsplit];
    auto first = ct.perm.begin() + off;
    if (role[t] == ROLE_DOMAIN) {
      // interface hyperplane x_d = floor((lo+hi)/2): order D1 (below), D2 (above), I
      const int64_t m = mid2 >= 0 ? mid2 / 2 : -((-mid2 + 1) / 2);
      int n1 = 0, ni = 0, n2 = 0;
      for (int i = 0; i < sz; ++i) {
        const int64_t x = coords[first[i] * dim + dsplit];
        n1 += x < m; ni += x == m; n2 += x > m;
      }
      if (n1 > 0 && ni > 0 && n2 > 0) {
        tmp.clear();
        for (int i = 0; i < sz; ++i) if (coords[first[i] * dim + dsplit] < m) tmp.push_back(first[i]);
        for (int i = 0; i < sz; ++i) if (coords[first[i] * dim + dsplit] > m) tmp.push_back(first[i]);
        for (int i = 0; i < sz; ++i) if (coords[first[i] * dim + dsplit] == m) tmp.push_back(first[i]);
        std::copy(tmp.begin(), tmp.end(), first);
        const int s0 = add(off, n1 + n2, ct.level[t] + 1, t, ROLE_UNION, n1);
        const int s1 = add(off + n1 + n2, ni, ct.level[t] + 1, t, ROLE_OTHER, 0);
        ct.son0[t] = s0; ct.son1[t] = s1;
        continue;
      }
    }
    auto mid = std::stable_partition(first, first + sz, [&](int64_t idx) {
      return 2 * (int64_t)coords[idx * dim + dsplit] <= mid2;
    });
    const int n0 = (int)(mid - first);
    if (n0 <= 0 || n0 >= sz) throw H2Error(H2_ERR_ARG, "cluster cannot be split (duplicate points?)");
    const char rs = role[t] == ROLE_DOMAIN ? ROLE_DOMAIN : ROLE_OTHER;
    const int s0 = add(off, n0, ct.level[t] + 1, t, rs, 0);
    const int s1 = add(off + n0, sz - n0, ct.level[t] + 1, t, rs, 0);
    ct.son0[t] = s0; ct.son1[t] = s1;
  }
  ct.uni.assign(ct.offset.size(), 0);
  for (size_t t = 0; t < ct.offset.size(); ++t) ct.uni[t] = role[t] == ROLE_UNION && ct.son0[t] >= 0;
  ct.nc = (int)ct.offset.size();
  ct.depth = *std::max_element(ct.level.begin(), ct.level.end());
  ct.nlev = ct.depth + 1;
  // descendants of every cluster per level: contiguous id ranges (BFS order)
  ct.desc_lo.assign((size_t)ct.nc * ct.nlev, 0);
  ct.desc_hi.assign((size_t)ct.nc * ct.nlev, 0);
  for (int t = 0; t < ct.nc; ++t) {
    int a = t, b = t + 1;
    for (int lv = ct.level[t]; lv < ct.nlev; ++lv) {
      ct.desc_lo[(size_t)t * ct.nlev + lv] = a;
      ct.desc_hi[(size_t)t * ct.nlev + lv] = b;
      int na = -1, nb = -1;
      for (int c = a; c < b; ++c) {
        if (ct.son0[c] >= 0) {
          if (na < 0) na = ct.son0[c];
          nb = ct.son1[c] + 1;
        }
      }
      if (na < 0) { a = b = 0; } else { a = na; b = nb; }
    }
  }
}

// =============================================================== block tree
struct h2_btree_s {
  h2_ctx ctx;
  h2_ctree ct;
  double eta = 2.0;
  int nb = 0;
  std::vector<int> row, col, kind, parent, first, nsons;
  std::unordered_map<int64_t, int> index;
  Dev<int> d_row, d_col, d_kind, d_first, d_nsons;
  int find(int t, int s) const {
    auto it = index.find((int64_t)t * ct->nc + s);
    return it == index.end() ? -1 : it->second;
  }
};

static bool admissible(const h2_ctree_s &ct, int t, int s, double eta2) {
  int64_t dt = 0, ds = 0, dist = 0, gmax = 0;
  for (int d = 0; d < ct.dim; ++d) {
    const int64_t lt = ct.lo[t * ct.dim + d], ht = ct.hi[t * ct.dim + d];
    const int64_t ls = ct.lo[s * ct.dim + d], hs = ct.hi[s * ct.dim + d];
    dt += (ht - lt) * (ht - lt);
    ds += (hs - ls) * (hs - ls);
    const int64_t g = std::max<int64_t>(0, std::max(ls - ht, lt - hs));
    dist += g * g;
    gmax = std::max(gmax, g);
  }
  // at least two grid steps apart along some axis: no reach-one stencil couples the boxes
  if (gmax >= 2 && (double)std::max(dt, ds) <= eta2 * (double)dist) return true;
  // the two domains below one cut: the matrix and its Cholesky factor vanish there
  const int p = ct.parent[t];
  return t != s && p >= 0 && p == ct.parent[s] && ct.uni[p];
}

static void build_btree(h2_btree_s &bt) {
  const h2_ctree_s &ct = *bt.ct;
  const double eta2 = bt.eta * bt.eta;
  std::deque<int> q;
  auto add = [&](int t, int s, int par) {
    bt.row.push_back(t); bt.col.push_back(s); bt.parent.push_back(par);
    bt.kind.push_back(0); bt.first.push_back(-1); bt.nsons.push_back(0);
    q.push_back((int)bt.row.size() - 1);
  };
  add(0, 0, -1);
  while (!q.empty()) {
    const int b = q.front();
    q.pop_front();
    const int t = bt.row[b], s = bt.col[b];
    if (admissible(ct, t, s, eta2)) { bt.kind[b] = 1; continue; }
    const bool lt = ct.son0[t] < 0, ls = ct.son0[s] < 0;
    if (lt && ls) { bt.kind[b] = 2; continue; }
    bt.first[b] = (int)bt.row.size();
    int cnt = 0;
    const int ts[2] = {lt ? t : ct.son0[t], ct.son1[t]};
    const int ss[2] = {ls ? s : ct.son0[s], ct.son1[s]};
    for (int i = 0; i < (lt ? 1 : 2); ++i)
      for (int j = 0; j < (ls ? 1 : 2); ++j) { add(ts[i], ss[j], b); ++cnt; }
    bt.nsons[b] = cnt;
  }
  bt.nb = (int)bt.row.size();
  bt.index.reserve(bt.nb * 2);
  for (int b = 0; b < bt.nb; ++b) bt.index[(int64_t)bt.row[b] * ct.nc + bt.col[b]] = b;
}

// ================================================================= matrices
struct h2_csr_s {
  h2_ctx ctx;
  int64_t n = 0;
  Dev<int64_t> rp;
  Dev<int> ci;
  Dev<double> v;
};

struct TaskList {
  Dev<Task> d;
  Dev<int> aux;      // block lists referenced by tasks (offsets in the tasks)
  int count = 0;
  bool built = false;
};

struct h2_mat_s {
  h2_ctx ctx;
  hipStream_t stream = nullptr;   // own copy: destroy must not touch ctx (may be gone)
  h2_btree bt;
  bool lower = false;
  bool poisoned = false;
  bool busy = false;      // part of a launched, unfinished batch (h2_job)
  int nadm = 0, nnear = 0;
  std::vector<int> bslot, adm, nearb;
  std::vector<int> rowptr, rowidx, colptr, colidx, nrowptr, nrowidx, ncolptr, ncolidx;
  Dev<int> d_bslot, d_rowptr, d_rowidx, d_colptr, d_colidx, d_nrowptr, d_nrowidx, d_ncolptr,
      d_ncolidx;
  Dev<int> d_k[2], d_rho_m[2], d_wrho_m[2], d_wB_m[2], d_wnewk[2], d_bcols, d_err;
  Dev<double> d_leaf[2], d_E[2], d_rho[2], d_wrho[2], d_wB[2], d_wR[2], d_S, d_N, d_xh, d_yh, d_buf;
  Dev<double> d_pcg;   // PCG vectors and scalars
  Dev<unsigned long long> d_prof;
  Dev<double> d_flops, d_wscr;
  Dev<DevEnv> d_env;          // device copy of env read by the interpreter
  DevEnv env_uploaded{};
  bool env_valid = false;
  TaskList chol, prec, tinv, prec_inv;
  TaskList upd;           // the last batched update's list (storage reused: no frees)
  TaskList trsv[2];       // forward (L) and backward (L^*) substitution alone
  TaskList lrf, lrsolve;  // LR factorisation, R^{-1} L^{-1} r
  TaskList prod;          // Z += alpha X Y with X, Y read through d_env3[1], d_env3[2]
  Dev<DevEnv> d_env3;     // this matrix's env and the product operands' envs
  double prod_alpha = 0.0;  // alpha the product task list was planned with
  bool inverse = false;   // holds G ~ L^{-1} (h2_tri_invert) instead of a factor L
  bool lr = false;        // holds the LR factors (h2_lr)
  // threads per workgroup of the substitution launches by column count
  // (h2_autotune_precond, h2_precond_config; 0: the default)
  int prec_nt[BC + 1] = {};
  DevEnv env{};
};

// Device copies of the tree tables, made when the first matrix needs them.
static void trees_to_device(h2_btree_s &bt, hipStream_t s) {
  h2_ctree_s &ct = *bt.ct;
  if (!ct.d_offset.p) {
    ct.d_perm.upload(ct.perm, s);
    ct.d_offset.upload(ct.offset, s); ct.d_size.upload(ct.size, s);
    ct.d_level.upload(ct.level, s); ct.d_son0.upload(ct.son0, s);
    ct.d_son1.upload(ct.son1, s); ct.d_parent.upload(ct.parent, s);
    ct.d_desc_lo.upload(ct.desc_lo, s); ct.d_desc_hi.upload(ct.desc_hi, s);
  }
  if (!bt.d_row.p) {
    bt.d_row.upload(bt.row, s); bt.d_col.upload(bt.col, s); bt.d_kind.upload(bt.kind, s);
    bt.d_first.upload(bt.first, s); bt.d_nsons.upload(bt.nsons, s);
  }
}

static void mat_alloc(h2_mat_s &m) {
  const h2_ctree_s &ct = *m.bt->ct;
  const size_t nc = ct.nc;
  hipStream_t s = m.ctx->stream;
  for (int side = 0; side < 2; ++side) {
    m.d_k[side].alloc_on(nc, s); m.d_k[side].zero(s);
    m.d_rho_m[side].alloc_on(nc, s); m.d_rho_m[side].zero(s);
    m.d_wrho_m[side].alloc_on(nc, s); m.d_wB_m[side].alloc_on(nc, s); m.d_wnewk[side].alloc_on(nc, s);
    m.d_leaf[side].alloc_on(nc * LS * KC, s);
    m.d_E[side].alloc_on(nc * KC * KC, s);
    m.d_rho[side].alloc_on(nc * KC * KC, s);
    m.d_wrho[side].alloc_on(nc * KM * KM, s);
    m.d_wB[side].alloc_on(nc * KM * KM, s);
    m.d_wR[side].alloc_on(nc * KM * KM, s);
  }
  m.d_S.alloc_on((size_t)std::max(m.nadm, 1) * KC * KC, s);
  m.d_N.alloc_on((size_t)std::max(m.nnear, 1) * LS * LS, s);
  m.d_xh.alloc_on(nc * KC * BC, s);
  m.d_yh.alloc_on(nc * KC * BC, s);
  m.d_buf.alloc_on((size_t)NBUF * ct.n * BC, s);
  m.d_bcols.alloc_on(NBUF, s); m.d_bcols.zero(s);
  m.d_err.alloc_on(4, s); m.d_err.zero(s);
  m.d_flops.alloc_on(1 + NWAVE, s); m.d_flops.zero(s);
  m.d_wscr.alloc_on((size_t)NWAVE * WGLOB, s);
}

// Device bytes a matrix holds now: storage, work areas, task lists, PCG
// vectors (the tree tables, shared by all matrices of a tree, excluded).
static size_t mat_bytes_now(const h2_mat_s &m) {
  size_t b = 0;
  auto add = [&](const auto &d) { b += d.n * sizeof(*d.p); };
  add(m.d_bslot); add(m.d_rowptr); add(m.d_rowidx); add(m.d_colptr); add(m.d_colidx);
  add(m.d_nrowptr); add(m.d_nrowidx); add(m.d_ncolptr); add(m.d_ncolidx);
  for (int side = 0; side < 2; ++side) {
    add(m.d_k[side]); add(m.d_rho_m[side]); add(m.d_wrho_m[side]); add(m.d_wB_m[side]); add(m.d_wnewk[side]);
    add(m.d_leaf[side]); add(m.d_E[side]); add(m.d_rho[side]); add(m.d_wrho[side]); add(m.d_wB[side]);
    add(m.d_wR[side]);
  }
  add(m.d_bcols); add(m.d_err); add(m.d_S); add(m.d_N); add(m.d_xh); add(m.d_yh); add(m.d_buf);
  add(m.d_pcg); add(m.d_prof); add(m.d_flops); add(m.d_wscr); add(m.d_env); add(m.d_env3);
  for (const TaskList *tl : {&m.chol, &m.prec, &m.tinv, &m.prec_inv, &m.upd, &m.trsv[0], &m.trsv[1], &m.lrf,
                             &m.lrsolve, &m.prod}) {
    add(tl->d);
    add(tl->aux);
  }
  return b;
}

// Device bytes h2_mat_from_csr allocates for a block tree (storage, work
// areas and block lists; no task lists yet): the sizes of mat_alloc and
// mat_lists.
static size_t mat_bytes_planned(const h2_btree_s &bt, bool lower) {
  const h2_ctree_s &ct = *bt.ct;
  const size_t nc = ct.nc;
  size_t nadm = 0, nnear = 0;
  for (int b = 0; b < bt.nb; ++b) {
    if (bt.kind[b] == 0) continue;
    const int t = bt.row[b], s = bt.col[b];
    if (lower && !(t == s || ct.offset[t] > ct.offset[s])) continue;
    (bt.kind[b] == 1 ? nadm : nnear)++;
  }
  size_t ints = bt.nb + 4 * (nc + 1) + 2 * nadm + 2 * nnear + 2 * 5 * nc + NBUF + 4;
  size_t dbl = 2 * (nc * LS * KC + 2 * nc * KC * KC + 3 * nc * KM * KM) + std::max<size_t>(nadm, 1) * KC * KC +
               std::max<size_t>(nnear, 1) * LS * LS + 2 * nc * KC * BC + (size_t)NBUF * ct.n * BC + 1 + NWAVE +
               (size_t)NWAVE * WGLOB;
  return ints * sizeof(int) + dbl * sizeof(double);
}

static void mat_lists(h2_mat_s &m) {
  const h2_btree_s &bt = *m.bt;
  const h2_ctree_s &ct = *bt.ct;
  m.bslot.assign(bt.nb, -1);
  m.adm.clear(); m.nearb.clear();
  for (int b = 0; b < bt.nb; ++b) {
    if (bt.kind[b] == 0) continue;
    const int t = bt.row[b], s = bt.col[b];
    if (m.lower && !(t == s || ct.offset[t] > ct.offset[s])) continue;
    if (bt.kind[b] == 1) { m.bslot[b] = (int)m.adm.size(); m.adm.push_back(b); }
    else { m.bslot[b] = (int)m.nearb.size(); m.nearb.push_back(b); }
  }
  m.nadm = (int)m.adm.size();
  m.nnear = (int)m.nearb.size();
  auto csr = [&](const std::vector<int> &blocks, bool byrow, std::vector<int> &ptr, std::vector<int> &idx) {
    ptr.assign(ct.nc + 1, 0);
    for (int b : blocks) ptr[(byrow ? bt.row[b] : bt.col[b]) + 1]++;
    for (int c = 0; c < ct.nc; ++c) ptr[c + 1] += ptr[c];
    idx.assign(blocks.size(), 0);
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (int b : blocks) idx[fill[byrow ? bt.row[b] : bt.col[b]]++] = b;   // blocks ascend by id
  };
  csr(m.adm, true, m.rowptr, m.rowidx);
  csr(m.adm, false, m.colptr, m.colidx);
  csr(m.nearb, true, m.nrowptr, m.nrowidx);
  csr(m.nearb, false, m.ncolptr, m.ncolidx);
  hipStream_t s = m.ctx->stream;
  m.d_bslot.upload(m.bslot, s);
  m.d_rowptr.upload(m.rowptr, s); m.d_rowidx.upload(m.rowidx, s);
  m.d_colptr.upload(m.colptr, s); m.d_colidx.upload(m.colidx, s);
  m.d_nrowptr.upload(m.nrowptr, s); m.d_nrowidx.upload(m.nrowidx, s);
  m.d_ncolptr.upload(m.ncolptr, s); m.d_ncolidx.upload(m.ncolidx, s);
}

static void mat_env(h2_mat_s &m) {
  const h2_ctree_s &ct = *m.bt->ct;
  const h2_btree_s &bt = *m.bt;
  DevEnv &e = m.env;
  e.n = (int)ct.n; e.nc = ct.nc; e.depth = ct.depth; e.nlev = ct.nlev;
  e.rank_cap = KC; e.mode = 0; e.eps = 0.0;
  e.offset = ct.d_offset.p; e.size = ct.d_size.p; e.son0 = ct.d_son0.p; e.son1 = ct.d_son1.p;
  e.parent = ct.d_parent.p; e.level = ct.d_level.p; e.desc_lo = ct.d_desc_lo.p; e.desc_hi = ct.d_desc_hi.p;
  e.brow = bt.d_row.p; e.bcol = bt.d_col.p; e.bkind = bt.d_kind.p; e.bfirst = bt.d_first.p;
  e.bnsons = bt.d_nsons.p; e.bslot = m.d_bslot.p;
  e.rowptr = m.d_rowptr.p; e.rowidx = m.d_rowidx.p; e.colptr = m.d_colptr.p; e.colidx = m.d_colidx.p;
  e.nrowptr = m.d_nrowptr.p; e.nrowidx = m.d_nrowidx.p; e.ncolptr = m.d_ncolptr.p; e.ncolidx = m.d_ncolidx.p;
  for (int side = 0; side < 2; ++side) {
    e.k[side] = m.d_k[side].p; e.leaf[side] = m.d_leaf[side].p; e.E[side] = m.d_E[side].p;
    e.rho[side] = m.d_rho[side].p; e.rho_m[side] = m.d_rho_m[side].p;
    e.wrho[side] = m.d_wrho[side].p; e.wrho_m[side] = m.d_wrho_m[side].p;
    e.wB[side] = m.d_wB[side].p; e.wB_m[side] = m.d_wB_m[side].p;
    e.wR[side] = m.d_wR[side].p; e.wnewk[side] = m.d_wnewk[side].p;
  }
  e.S = m.d_S.p; e.N = m.d_N.p; e.xh = m.d_xh.p; e.yh = m.d_yh.p;
  for (int i = 0; i < NBUF; ++i) e.buf[i] = m.d_buf.p + (size_t)i * ct.n * BC;
  e.bcols = m.d_bcols.p; e.err = m.d_err.p; e.flops = m.d_flops.p; e.wscr = m.d_wscr.p;
}

// ================================================================== planner
// Turns the recursive algorithms into task lists; see tasks.hip for the
// meaning of each task.  The recursion follows Section 3 (product, block
// substitution, LR/Cholesky) and Section 6 (Cases 1 and 2).
struct Planner {
  const h2_mat_s &M;
  const h2_ctree_s &ct;
  const h2_btree_s &bt;
  std::vector<Task> &T;
  std::vector<int> aux;
  Planner(const h2_mat_s &m, std::vector<Task> &t) : M(m), ct(*m.bt->ct), bt(*m.bt), T(t) {}

  // environment of the next emitted tasks: 0 = the target matrix; the
  // product of three matrices reads X through 1 and Y through 2 (ex, ey)
  int env = 0, ex = 0, ey = 0;

  void emit(int op, int a = 0, int b = 0, int c = 0, int d = 0, int e_ = 0, int f = 0, int g = 0,
            int h = 0, double alpha = 0.0, double beta = 0.0) {
    Task k{};
    k.op = op;
    k.env = env;
    k.i[0] = a; k.i[1] = b; k.i[2] = c; k.i[3] = d; k.i[4] = e_; k.i[5] = f; k.i[6] = g; k.i[7] = h;
    k.alpha = alpha; k.beta = beta;
    T.push_back(k);
  }
  int find(int t, int s) const {
    const int b = bt.find(t, s);
    if (b < 0) throw H2Error(H2_ERR_ARG, "internal: block not in tree");
    return b;
  }
  bool leaf(int t) const { return ct.son0[t] < 0; }
  std::vector<int> sons_plus(int t) const {
    if (leaf(t)) return {t};
    return {ct.son0[t], ct.son1[t]};
  }
  static int TU(int p) { return B_T0U + 2 * p; }
  static int TV(int p) { return B_T0V + 2 * p; }

  void bapply(int b, int trans, int bin, int bout, double alpha, double beta) {
    emit(OP_BAPPLY, b, trans, bin, bout, 0, 0, 0, 0, alpha, beta);
  }
  void addlr(int b, int bu, int bv) { emit(OP_ADDLR, b, bu, bv); }

  // H^2 substitution: one pass over the clusters and blocks of the subtree
  // (forward transformations of solved clusters reused, coupling sums pushed
  // down the unsolved part).
  void leaves_of(int b, std::vector<int> &out) const {
    if (bt.kind[b] != 0) { out.push_back(b); return; }
    const int t = bt.row[b], s = bt.col[b];
    for (int t2 : sons_plus(t))
      for (int s2 : sons_plus(s)) leaves_of(find(t2, s2), out);
  }
  // Leaves of block (c2, c1) grouped by the cluster they update (row cluster
  // for trans = 0, column cluster for trans = 1): aux holds the group start
  // offsets, then per group {cluster, count, blocks...}.  Returns the offset
  // of the start table; ng receives the number of groups.
  int cross_groups(int c2, int c1, int trans, int &ng) {
    std::vector<int> lv;
    leaves_of(find(c2, c1), lv);
    std::vector<int> tgt;
    std::vector<std::vector<int>> grp;
    std::unordered_map<int, int> where;
    for (int b : lv) {
      const int t = trans ? bt.col[b] : bt.row[b];
      auto it = where.find(t);
      if (it == where.end()) { where[t] = (int)tgt.size(); tgt.push_back(t); grp.emplace_back(); it = where.find(t); }
      grp[it->second].push_back(b);
    }
    ng = (int)tgt.size();
    const int off = (int)aux.size();
    aux.resize(aux.size() + ng);
    for (int g = 0; g < ng; ++g) {
      aux[off + g] = (int)aux.size();
      aux.push_back(tgt[g]);
      aux.push_back((int)grp[g].size());
      for (int b : grp[g]) aux.push_back(b);
    }
    return off;
  }
  void sv_rec(int c, int buf, int trans, bool top) {
    if (leaf(c)) { emit(OP_SV_LEAF, find(c, c), buf, trans); return; }
    const int c1 = ct.son0[c], c2 = ct.son1[c];
    if (!top) emit(OP_SV_PUSH, c, buf, trans);
    sv_rec(trans ? c2 : c1, buf, trans, false);
    int ng;
    const int off = cross_groups(c2, c1, trans, ng);
    emit(OP_SV_CROSS, off, ng, buf, trans);
    sv_rec(trans ? c1 : c2, buf, trans, false);
    if (!top) emit(OP_SV_UP, c, buf, trans);
  }
  void fsolve_h2(int c, int buf) { emit(OP_SV_ZERO, c, buf, 0); sv_rec(c, buf, 0, true); }
  void bsolve_h2(int c, int buf) { emit(OP_SV_ZERO, c, buf, 1); sv_rec(c, buf, 1, true); }

  void fsolve(int c, int buf) {
    if (leaf(c)) { emit(OP_TRSV, find(c, c), buf, 0); return; }
    const int c1 = ct.son0[c], c2 = ct.son1[c];
    fsolve(c1, buf);
    bapply(find(c2, c1), 0, buf, buf, -1.0, 1.0);
    fsolve(c2, buf);
  }
  void bsolve(int c, int buf) {
    if (leaf(c)) { emit(OP_TRSV, find(c, c), buf, 1); return; }
    const int c1 = ct.son0[c], c2 = ct.son1[c];
    bsolve(c2, buf);
    bapply(find(c2, c1), 1, buf, buf, -1.0, 1.0);
    bsolve(c1, buf);
  }

  // Z(t, r) += alpha X(t, s) Y(r, s)^* with X, Y, Z blocks of the factor.
  void mm(int t, int s, int r, double alpha, int tmp, int tT, int rT) {
    const int bX = find(t, s), bY = find(r, s);
    if (bt.kind[bX] == 0 && bt.kind[bY] == 0) {
      const auto ts = sons_plus(t), ss = sons_plus(s), rs = sons_plus(r);
      if (tmp >= 0) {
        for (int s2 : ss) for (int t2 : ts) for (int r2 : rs) mm(t2, s2, r2, alpha, tmp, tT, rT);
        return;
      }
      const int bZ = find(t, r);
      if (bt.kind[bZ] == 0) {
        for (int s2 : ss)
          for (int t2 : ts)
            for (int r2 : rs) {
              if (ct.offset[t2] < ct.offset[r2]) continue;   // above the diagonal
              mm(t2, s2, r2, alpha, -1, 0, 0);
            }
      } else if (bt.kind[bZ] == 2) {
        const int ns = ct.size[s];
        for (int c0 = 0; c0 < ns; c0 += BC) {
          const int nc = std::min(BC, ns - c0);
          emit(OP_IDENT, s, B_I, c0, nc);
          bapply(bX, 0, B_I, B_A, 1.0, 0.0);
          bapply(bY, 0, B_I, B_B, 1.0, 0.0);
          emit(OP_NEAR_ADD, bZ, B_A, B_B, 0, 0, 0, 0, 0, alpha);
        }
      } else {
        std::vector<std::pair<int, int>> pairs;
        for (int t2 : ts) for (int r2 : rs) pairs.push_back({t2, r2});
        for (size_t p = 0; p < pairs.size(); ++p) emit(OP_TEMP_INIT, TU((int)p), TV((int)p), t, r);
        for (int s2 : ss)
          for (int t2 : ts)
            for (int r2 : rs) {
              int p = 0;
              while (pairs[p].first != t2 || pairs[p].second != r2) ++p;
              mm(t2, s2, r2, alpha, p, t2, r2);
            }
        emit(OP_ADDLR_ACC, bZ, (int)pairs.size());
      }
      return;
    }
    // Case 2: a factor is a leaf -> low-rank emission (U, V)
    if (bt.kind[bY] == 1) {
      emit(OP_EXPAND, 1, s, B_W);
      bapply(bX, 0, B_W, B_A, 1.0, 0.0);
      emit(OP_RMUL_S, B_A, B_U, bY, 1, t, 0, 0, 0, alpha);
      emit(OP_EXPAND, 0, r, B_V);
    } else if (bt.kind[bX] == 1) {
      emit(OP_EXPAND, 0, t, B_A);
      emit(OP_RMUL_S, B_A, B_U, bX, 0, t, 0, 0, 0, alpha);
      emit(OP_EXPAND, 1, s, B_W);
      bapply(bY, 0, B_W, B_V, 1.0, 0.0);
    } else if (bt.kind[bX] == 2) {
      emit(OP_COPY_NEAR, bX, B_U, 0, 0, 0, 0, 0, 0, alpha);
      emit(OP_IDENT, s, B_I, 0, ct.size[s]);
      bapply(bY, 0, B_I, B_V, 1.0, 0.0);
    } else {
      emit(OP_IDENT, s, B_I, 0, ct.size[s]);
      bapply(bX, 0, B_I, B_U, alpha, 0.0);
      emit(OP_COPY_NEAR, bY, B_V, 0, 0, 0, 0, 0, 0, 1.0);
    }
    if (tmp >= 0) {
      emit(OP_TEMP_ADD, TU(tmp), TV(tmp), t, r, B_U, B_V, tT, rT);
    } else {
      const int bZ = find(t, r);
      if (bt.kind[bZ] == 2) emit(OP_NEAR_ADD, bZ, B_U, B_V, 0, 0, 0, 0, 0, 1.0);
      else addlr(bZ, B_U, B_V);
    }
  }

  // X L_cc^* = Y on block b = (r, c), in place.
  void rsolve(int c, int b) {
    const int r = bt.row[b];
    if (bt.kind[b] == 0) {
      if (leaf(c)) {
        for (int r2 : sons_plus(r)) rsolve(c, find(r2, c));
        return;
      }
      const int c1 = ct.son0[c], c2 = ct.son1[c];
      const auto rs = sons_plus(r);
      for (int r2 : rs) rsolve(c1, find(r2, c1));
      for (int r2 : rs) mm(r2, c1, c2, -1.0, -1, 0, 0);
      for (int r2 : rs) rsolve(c2, find(r2, c2));
    } else if (bt.kind[b] == 2) {
      emit(OP_TRSM, b, find(c, c));
    } else {
      emit(OP_EXPAND, 1, c, B_W);
      emit(OP_COPY, B_W, B_WP, c);
      fsolve(c, B_WP);
      emit(OP_SUB, B_WP, B_W, B_V, c);
      emit(OP_EXPAND, 0, r, B_A);
      emit(OP_RMUL_S, B_A, B_U, b, 0, r, 0, 0, 0, 1.0);
      addlr(b, B_U, B_V);
    }
  }

  // Z(t, r) += alpha X(t, s) Y(s, r) with X = block (t, s) and Y = block
  // (s, r) of a lower triangular matrix, all three strictly below the
  // diagonal: the recursion of mm with the second factor used as stored
  // instead of transposed.
  void mm_n(int t, int s, int r, double alpha, int tmp, int tT, int rT) {
    const int bX = find(t, s), bY = find(s, r);
    if (bt.kind[bX] == 0 && bt.kind[bY] == 0) {
      const auto ts = sons_plus(t), ss = sons_plus(s), rs = sons_plus(r);
      if (tmp >= 0) {
        for (int s2 : ss) for (int t2 : ts) for (int r2 : rs) mm_n(t2, s2, r2, alpha, tmp, tT, rT);
        return;
      }
      const int bZ = find(t, r);
      if (bt.kind[bZ] == 0) {
        for (int s2 : ss) for (int t2 : ts) for (int r2 : rs) mm_n(t2, s2, r2, alpha, -1, 0, 0);
      } else if (bt.kind[bZ] == 2) {
        const int ns = ct.size[s];
        for (int c0 = 0; c0 < ns; c0 += BC) {
          const int nc = std::min(BC, ns - c0);
          emit(OP_IDENT, s, B_I, c0, nc);
          env = ex; bapply(bX, 0, B_I, B_A, 1.0, 0.0);
          env = ey; bapply(bY, 1, B_I, B_B, 1.0, 0.0);
          env = 0;
          emit(OP_NEAR_ADD, bZ, B_A, B_B, 0, 0, 0, 0, 0, alpha);
        }
      } else {
        std::vector<std::pair<int, int>> pairs;
        for (int t2 : ts) for (int r2 : rs) pairs.push_back({t2, r2});
        for (size_t p = 0; p < pairs.size(); ++p) emit(OP_TEMP_INIT, TU((int)p), TV((int)p), t, r);
        for (int s2 : ss)
          for (int t2 : ts)
            for (int r2 : rs) {
              int p = 0;
              while (pairs[p].first != t2 || pairs[p].second != r2) ++p;
              mm_n(t2, s2, r2, alpha, p, t2, r2);
            }
        emit(OP_ADDLR_ACC, bZ, (int)pairs.size());
      }
      return;
    }
    if (bt.kind[bY] == 1) {          // Y = V_s S W_r^*: U = alpha (X V_s) S, V = W_r
      env = ey; emit(OP_EXPAND, 0, s, B_W);
      env = ex; bapply(bX, 0, B_W, B_A, 1.0, 0.0);
      env = ey; emit(OP_RMUL_S, B_A, B_U, bY, 0, t, 0, 0, 0, alpha);
      emit(OP_EXPAND, 1, r, B_V);
    } else if (bt.kind[bX] == 1) {   // X = V_t S W_s^*: U = alpha V_t S, V = Y^* W_s
      env = ex; emit(OP_EXPAND, 0, t, B_A);
      emit(OP_RMUL_S, B_A, B_U, bX, 0, t, 0, 0, 0, alpha);
      emit(OP_EXPAND, 1, s, B_W);
      env = ey; bapply(bY, 1, B_W, B_V, 1.0, 0.0);
    } else if (bt.kind[bX] == 2) {   // U = alpha N_X, V = Y^* expanded
      env = ex; emit(OP_COPY_NEAR, bX, B_U, 0, 0, 0, 0, 0, 0, alpha);
      env = 0; emit(OP_IDENT, s, B_I, 0, ct.size[s]);
      env = ey; bapply(bY, 1, B_I, B_V, 1.0, 0.0);
    } else {                         // U = alpha X expanded, V = N_Y^*
      emit(OP_IDENT, s, B_I, 0, ct.size[s]);
      env = ex; bapply(bX, 0, B_I, B_U, alpha, 0.0);
      env = ey; emit(OP_COPY_NEAR, bY, B_V, 1, 0, 0, 0, 0, 0, 1.0);
    }
    env = 0;
    if (tmp >= 0) {
      emit(OP_TEMP_ADD, TU(tmp), TV(tmp), t, r, B_U, B_V, tT, rT);
    } else {
      const int bZ = find(t, r);
      if (bt.kind[bZ] == 2) emit(OP_NEAR_ADD, bZ, B_U, B_V, 0, 0, 0, 0, 0, 1.0);
      else addlr(bZ, B_U, B_V);
    }
  }

  // ---- LR factorisation (Section 3) of a full-storage matrix in place:
  // unit lower L below the diagonal, R on and above it; no pivoting.
  // Vector solves with the factors of the diagonal block (c, c):
  // L_cc y = w (forward), R_cc^* y = w (forward), R_cc y = w (backward).
  void fsolve_unit(int c, int buf) {
    if (leaf(c)) { emit(OP_TRSV, find(c, c), buf, 0, TRI_L_UNIT); return; }
    const int c1 = ct.son0[c], c2 = ct.son1[c];
    fsolve_unit(c1, buf);
    bapply(find(c2, c1), 0, buf, buf, -1.0, 1.0);
    fsolve_unit(c2, buf);
  }
  void fsolve_radj(int c, int buf) {
    if (leaf(c)) { emit(OP_TRSV, find(c, c), buf, 0, TRI_R_ADJ); return; }
    const int c1 = ct.son0[c], c2 = ct.son1[c];
    fsolve_radj(c1, buf);
    bapply(find(c1, c2), 1, buf, buf, -1.0, 1.0);
    fsolve_radj(c2, buf);
  }
  void bsolve_upper(int c, int buf) {
    if (leaf(c)) { emit(OP_TRSV, find(c, c), buf, 0, TRI_R); return; }
    const int c1 = ct.son0[c], c2 = ct.son1[c];
    bsolve_upper(c2, buf);
    bapply(find(c1, c2), 0, buf, buf, -1.0, 1.0);
    bsolve_upper(c1, buf);
  }
  // L_cc X = Y on block b = (c, r), in place (block forward substitution).
  void lsolve_lr(int c, int b) {
    const int r = bt.col[b];
    if (bt.kind[b] == 0) {
      if (leaf(c)) {
        for (int r2 : sons_plus(r)) lsolve_lr(c, find(c, r2));
        return;
      }
      const int c1 = ct.son0[c], c2 = ct.son1[c];
      const auto rs = sons_plus(r);
      for (int r2 : rs) lsolve_lr(c1, find(c1, r2));
      for (int r2 : rs) mm_n(c2, c1, r2, -1.0, -1, 0, 0);
      for (int r2 : rs) lsolve_lr(c2, find(c2, r2));
    } else if (bt.kind[b] == 2) {
      emit(OP_TRSM, b, find(c, c), TRI_L_UNIT);
    } else {
      // L_cc^{-1} V_c S W_r^*, added as the update (L_cc^{-1} V_c - V_c)(W_r S^*)^*
      emit(OP_EXPAND, 0, c, B_W);
      emit(OP_COPY, B_W, B_WP, c);
      fsolve_unit(c, B_WP);
      emit(OP_SUB, B_WP, B_W, B_U, c);
      emit(OP_EXPAND, 1, r, B_A);
      emit(OP_RMUL_S, B_A, B_V, b, 1, r, 0, 0, 0, 1.0);
      addlr(b, B_U, B_V);
    }
  }
  // X R_cc = Y on block b = (r, c), in place.
  void rsolve_lr(int c, int b) {
    const int r = bt.row[b];
    if (bt.kind[b] == 0) {
      if (leaf(c)) {
        for (int r2 : sons_plus(r)) rsolve_lr(c, find(r2, c));
        return;
      }
      const int c1 = ct.son0[c], c2 = ct.son1[c];
      const auto rs = sons_plus(r);
      for (int r2 : rs) rsolve_lr(c1, find(r2, c1));
      for (int r2 : rs) mm_n(r2, c1, c2, -1.0, -1, 0, 0);
      for (int r2 : rs) rsolve_lr(c2, find(r2, c2));
    } else if (bt.kind[b] == 2) {
      emit(OP_TRSM, b, find(c, c), TRI_R_ADJ);
    } else {
      // V_r S W_c^* R_cc^{-1} = V_r S (R_cc^{-*} W_c)^*, added as the update
      // (V_r S)(R_cc^{-*} W_c - W_c)^*
      emit(OP_EXPAND, 1, c, B_W);
      emit(OP_COPY, B_W, B_WP, c);
      fsolve_radj(c, B_WP);
      emit(OP_SUB, B_WP, B_W, B_V, c);
      emit(OP_EXPAND, 0, r, B_A);
      emit(OP_RMUL_S, B_A, B_U, b, 0, r, 0, 0, 0, 1.0);
      addlr(b, B_U, B_V);
    }
  }
  void lr(int t) {
    if (leaf(t)) { emit(OP_GETRF, find(t, t), t); return; }
    const int t1 = ct.son0[t], t2 = ct.son1[t];
    lr(t1);
    lsolve_lr(t1, find(t1, t2));
    rsolve_lr(t1, find(t2, t1));
    mm_n(t2, t1, t2, -1.0, -1, 0, 0);
    lr(t2);
  }

  // buf|_c <- G_cc buf|_c (trans: G_cc^* buf|_c) in place, G lower
  // triangular: dense lower triangle on a leaf, otherwise the sons' diagonal
  // blocks and the block (c2, c1); the part that is read later is updated
  // last.
  void trmv(int c, int buf, int trans) {
    if (leaf(c)) { emit(OP_TRMV, find(c, c), buf, trans); return; }
    const int c1 = ct.son0[c], c2 = ct.son1[c];
    if (!trans) {
      trmv(c2, buf, 0);
      bapply(find(c2, c1), 0, buf, buf, 1.0, 1.0);
      trmv(c1, buf, 0);
    } else {
      trmv(c1, buf, 1);
      bapply(find(c2, c1), 1, buf, buf, 1.0, 1.0);
      trmv(c2, buf, 1);
    }
  }

  // X(r, c) <- X(r, c) G_cc in place on block b = (r, c), the diagonal
  // block (c, c) already inverted.  Sons c1, c2 of c split X into [X1 X2]:
  // X1 <- X1 G_11, X1 += X2 G_21 (X2 still untouched), X2 <- X2 G_22.
  void rmul_tri(int c, int b) {
    const int r = bt.row[b];
    if (bt.kind[b] == 0) {
      if (leaf(c)) {
        for (int r2 : sons_plus(r)) rmul_tri(c, find(r2, c));
        return;
      }
      const int c1 = ct.son0[c], c2 = ct.son1[c];
      const auto rs = sons_plus(r);
      for (int r2 : rs) rmul_tri(c1, find(r2, c1));
      for (int r2 : rs) mm_n(r2, c2, c1, 1.0, -1, 0, 0);
      for (int r2 : rs) rmul_tri(c2, find(r2, c2));
    } else if (bt.kind[b] == 2) {
      emit(OP_NEAR_TRMUL, b, find(c, c), 1);          // N_b <- N_b G_cc
    } else {
      // V_r S W_c^* G_cc = V_r S (G_cc^* W_c)^*, added as the update
      // (V_r S)(G_cc^* W_c - W_c)^* because W_c is shared
      emit(OP_EXPAND, 1, c, B_W);
      emit(OP_COPY, B_W, B_WP, c);
      trmv(c, B_WP, 1);
      emit(OP_SUB, B_WP, B_W, B_V, c);
      emit(OP_EXPAND, 0, r, B_A);
      emit(OP_RMUL_S, B_A, B_U, b, 0, r, 0, 0, 0, 1.0);
      addlr(b, B_U, B_V);
    }
  }

  // Y(c, r) <- G_cc Y(c, r) in place on block b = (c, r).  Sons split Y into
  // [Y1; Y2]: Y2 <- G_22 Y2, Y2 += G_21 Y1 (Y1 still untouched),
  // Y1 <- G_11 Y1.
  void lmul_tri(int c, int b) {
    const int r = bt.col[b];
    if (bt.kind[b] == 0) {
      if (leaf(c)) {
        for (int r2 : sons_plus(r)) lmul_tri(c, find(c, r2));
        return;
      }
      const int c1 = ct.son0[c], c2 = ct.son1[c];
      const auto rs = sons_plus(r);
      for (int r2 : rs) lmul_tri(c2, find(c2, r2));
      for (int r2 : rs) mm_n(c2, c1, r2, 1.0, -1, 0, 0);
      for (int r2 : rs) lmul_tri(c1, find(c1, r2));
    } else if (bt.kind[b] == 2) {
      emit(OP_NEAR_TRMUL, b, find(c, c), 0);          // N_b <- G_cc N_b
    } else {
      // G_cc V_c S W_r^*, added as the update (G_cc V_c - V_c)(W_r S^*)^*
      emit(OP_EXPAND, 0, c, B_W);
      emit(OP_COPY, B_W, B_WP, c);
      trmv(c, B_WP, 0);
      emit(OP_SUB, B_WP, B_W, B_U, c);
      emit(OP_EXPAND, 1, r, B_A);
      emit(OP_RMUL_S, B_A, B_V, b, 1, r, 0, 0, 0, 1.0);
      addlr(b, B_U, B_V);
    }
  }

  void neg(int b) {
    std::vector<int> lv;
    leaves_of(b, lv);
    const int off = (int)aux.size();
    for (int l : lv) aux.push_back(l);
    emit(OP_NEG, off, (int)lv.size());
  }

  // Triangular inverse (the inversion remark at the end of Section 6 with
  // A_12 = 0): C_11 = A_11^{-1}, C_22 = A_22^{-1}, C_21 = -C_22 A_21 C_11,
  // the last formed in place on the block (c2, c1).
  void tinv(int c) {
    if (leaf(c)) { emit(OP_TRTRI, find(c, c)); return; }
    const int c1 = ct.son0[c], c2 = ct.son1[c];
    const int b = find(c2, c1);
    tinv(c1);
    rmul_tri(c1, b);
    tinv(c2);
    lmul_tri(c2, b);
    neg(b);
  }

  void chol(int t) {
    if (leaf(t)) { emit(OP_POTRF, find(t, t), t); return; }
    const int t1 = ct.son0[t], t2 = ct.son1[t];
    chol(t1);
    rsolve(t1, find(t2, t1));
    mm(t2, t1, t2, -1.0, -1, 0, 0);
    chol(t2);
  }
};

static void upload_tasks(h2_mat_s &m, TaskList &tl, const std::vector<Task> &tasks,
                         const std::vector<int> &aux) {
  (void)m;
  tl.d.alloc_on(tasks.size(), m.stream);
  if (!tasks.empty())
    HIPCHK(hipMemcpy(tl.d.p, tasks.data(), tasks.size() * sizeof(Task), hipMemcpyHostToDevice));
  tl.aux.alloc_on(aux.size(), m.stream);
  if (!aux.empty())
    HIPCHK(hipMemcpy(tl.aux.p, aux.data(), aux.size() * sizeof(int), hipMemcpyHostToDevice));
  tl.count = (int)tasks.size();
  tl.built = true;
}

// As upload_tasks, but keeps the device arrays when they are large enough:
// freeing device memory would wait for every stream of the device.
static void upload_tasks_reuse(TaskList &tl, const std::vector<Task> &tasks, const std::vector<int> &aux) {
  if (tl.d.n < tasks.size()) tl.d.alloc(tasks.size());
  if (!tasks.empty())
    HIPCHK(hipMemcpy(tl.d.p, tasks.data(), tasks.size() * sizeof(Task), hipMemcpyHostToDevice));
  if (tl.aux.n < aux.size()) tl.aux.alloc(aux.size());
  if (!aux.empty())
    HIPCHK(hipMemcpy(tl.aux.p, aux.data(), aux.size() * sizeof(int), hipMemcpyHostToDevice));
  tl.count = (int)tasks.size();
  tl.built = true;
}

static void set_trunc(h2_mat_s &m, const h2_trunc *tr) {
  if (!tr) {
    m.env.eps = 0.0; m.env.mode = 2; m.env.rank_cap = KC; m.env.prec = 0; m.env.acc = 0; m.env.lvq = 1.0;
    return;
  }
  REQUIRE(tr->mode >= 0 && tr->mode <= 2, "truncation mode must be 0, 1 or 2");
  REQUIRE(tr->rank_cap >= 1 && tr->rank_cap <= KC, "rank_cap must be in [1, H2_MAX_RANK]");
  REQUIRE(tr->eps >= 0.0 && std::isfinite(tr->eps), "eps must be finite and >= 0");
  REQUIRE(tr->precision == H2_PREC_FP64 || tr->precision == H2_PREC_MIXED || tr->precision == H2_PREC_MIXED_BF16,
          "precision must be 0, 1 or 2");
  REQUIRE(tr->accumulate == 0 || tr->accumulate == 1, "accumulate must be 0 or 1");
  REQUIRE(tr->level_factor >= 0.0 && tr->level_factor <= 1.0, "level_factor must be in [0, 1] (0 means 1)");
  m.env.eps = tr->eps; m.env.mode = tr->mode; m.env.rank_cap = tr->rank_cap; m.env.prec = tr->precision;
  m.env.acc = tr->accumulate;
  m.env.lvq = tr->level_factor == 0.0 ? 1.0 : tr->level_factor;
}

static bool g_lds_attr_set = false;

// Upload env when it changed since the last upload (blocking copy, so the
// host struct may change afterwards).
static void sync_env(h2_mat_s &m) {
  if (!m.d_env.p) m.d_env.alloc_on(1, m.stream);
  if (!m.env_valid || std::memcmp(&m.env_uploaded, &m.env, sizeof(DevEnv)) != 0) {
    HIPCHK(hipMemcpy(m.d_env.p, &m.env, sizeof(DevEnv), hipMemcpyHostToDevice));
    m.env_uploaded = m.env;
    m.env_valid = true;
  }
}

// nthreads: workgroup size of the launch (NT, or 256 for task lists whose
// kinds distribute work by the run-time wave count).
static void run_tasks(h2_mat_s &m, const TaskList &tl, int nthreads = NT, const DevEnv *d_envs = nullptr) {
  const Task *d_tasks = tl.d.p;
  const int count = tl.count;
  const size_t lds = LDS_TOTAL_DOUBLES * sizeof(double);
  sync_env(m);
  if (!d_envs) d_envs = m.d_env.p;
  if (!g_lds_attr_set) {
    HIPCHK(hipFuncSetAttribute((const void *)k_interp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    g_lds_attr_set = true;
  }
  const int seg = 1 << 24;
  for (int off = 0; off < count; off += seg) {
    const int cnt = std::min(seg, count - off);
    hipLaunchKernelGGL(k_interp, dim3(1), dim3(nthreads), lds, m.ctx->stream, d_tasks + off, cnt, d_envs,
                       (const int *)tl.aux.p);
    HIPCHK(hipGetLastError());
  }
}

static void check_device_error(h2_mat_s &m) {
  int err[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(err, m.d_err.p, 2 * sizeof(int), hipMemcpyDeviceToHost, m.ctx->stream));
  HIPCHK(hipStreamSynchronize(m.ctx->stream));
  if (err[0] != 0) {
    m.poisoned = true;
    char msg[160];
    if (err[0] == E_NOT_SPD) {
      snprintf(msg, sizeof msg, "leaf block of cluster %d is not positive definite", err[1]);
      throw H2Error(H2_ERR_NOT_SPD, msg);
    }
    if (err[0] == E_ZERO_PIVOT) {
      snprintf(msg, sizeof msg, "zero pivot in the LR factorisation of the leaf block of cluster %d", err[1]);
      throw H2Error(H2_ERR_ZERO_PIVOT, msg);
    }
    if (err[0] == E_RANK_CAP) {
      snprintf(msg, sizeof msg, "rank cap exceeded at cluster %d", err[1]);
      throw H2Error(H2_ERR_RANK_CAP, msg);
    }
    if (err[0] == E_SCRATCH) {
      snprintf(msg, sizeof msg, "internal: wave work area too small (%d doubles requested)", err[1]);
      throw H2Error(H2_ERR_STATE, msg);
    }
    snprintf(msg, sizeof msg, "device task failed (code %d, info %d)", err[0], err[1]);
    throw H2Error(H2_ERR_ARG, msg);
  }
}

static void require_ok(h2_mat m) {
  REQUIRE(m != nullptr, "null matrix");
  if (m->poisoned) throw H2Error(H2_ERR_STATE, "matrix poisoned by an earlier failure");
  REQUIRE(!m->busy, "matrix belongs to an unfinished batch (finish its job first)");
}

// Fixed device work area of h2_pcg_noalloc: the PCG vectors r, z, p, q,
// the partial sums of the dot products and the scalars of one system of at
// most H2_NOALLOC_MAX_N unknowns.  Every device the library runs on holds
// its own copy until the process ends; calls on one device share it.
constexpr size_t NOALLOC_DOUBLES = (size_t)4 * H2_NOALLOC_MAX_N + 512;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

// Device address of this device's copy of scratch (looked up once per
// device, with that device current; the host-side name of the array is not
// a device address).
static double *noalloc_scratch(int device) {
  static std::mutex mu;
  static std::unordered_map<int, double *> ptrs;
  std::lock_guard<std::mutex> lock(mu);
  auto it = ptrs.find(device);
  if (it != ptrs.end()) return it->second;
  int cur = -1;
  HIPCHK(hipGetDevice(&cur));
  if (cur != device) HIPCHK(hipSetDevice(device));
  void *ptr = nullptr;
  const hipError_t rc = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (cur != device) HIPCHK(hipSetDevice(cur));
  if (rc != hipSuccess || !ptr)
    throw H2Error(H2_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(rc));
  ptrs[device] = static_cast<double *>(ptr);
  return static_cast<double *>(ptr);
}

// Largest number of admissible leaves in one block row of the tree.
static int tree_csp(const h2_btree_s &bt) {
  std::vector<int> cnt(bt.ct->nc, 0);
  int mx = 0;
  for (int b = 0; b < bt.nb; ++b)
    if (bt.kind[b] == 1) mx = std::max(mx, ++cnt[bt.row[b]]);
  return mx;
}

// Trees with block rows of more than 64 admissible leaves (the weight
// stacks then take several 64-block metadata chunks) are refused by every
// call that runs local updates: the one such workload tried, the
// domain-decomposition tree of the 256 x 256 grid at eta 4 (89 blocks in a
// row, depth 22), did not finish its factorisation on the GPU and the cause
// is not known.
constexpr int VALIDATED_CSP = 64;
static void require_validated_tree(const h2_mat_s &m) {
  const int csp = tree_csp(*m.bt);
  if (csp > VALIDATED_CSP)
    throw H2Error(H2_ERR_ARG, "block tree with " + std::to_string(csp) +
                                  " admissible blocks in one block row: updates on trees with more than " +
                                  std::to_string(VALIDATED_CSP) + " per row are refused (not validated)");
}

static int grid_for(long work) {
  long g = (work + 255) / 256;
  return (int)std::max<long>(1, std::min<long>(g, 4096));
}

// =================================================================== C ABI
// Stored values of the H^2 representation (leaf bases, transfer, coupling
// and nearfield matrices) and the largest ranks; reads the ranks back.
static int64_t mat_stored_values(h2_mat_s &m, int *kmax_row, int *kmax_col) {
  const h2_ctree_s &ct = *m.bt->ct;
  const h2_btree_s &bt = *m.bt;
  std::vector<int> k[2];
  for (int side = 0; side < 2; ++side) {
    k[side].resize(ct.nc);
    HIPCHK(hipMemcpyAsync(k[side].data(), m.d_k[side].p, ct.nc * sizeof(int), hipMemcpyDeviceToHost,
                          m.ctx->stream));
  }
  HIPCHK(hipStreamSynchronize(m.ctx->stream));
  int64_t vals = 0;
  for (int side = 0; side < 2; ++side)
    for (int c = 0; c < ct.nc; ++c) {
      if (ct.son0[c] < 0) vals += (int64_t)ct.size[c] * k[side][c];
      if (ct.parent[c] >= 0) vals += (int64_t)k[side][c] * k[side][ct.parent[c]];
    }
  for (int b : m.adm) vals += (int64_t)k[0][bt.row[b]] * k[1][bt.col[b]];
  for (int b : m.nearb) vals += (int64_t)ct.size[bt.row[b]] * ct.size[bt.col[b]];
  if (kmax_row) *kmax_row = *std::max_element(k[0].begin(), k[0].end());
  if (kmax_col) *kmax_col = *std::max_element(k[1].begin(), k[1].end());
  return vals;
}

extern "C" {

const char *h2_last_error(void) { return g_last_error.c_str(); }

h2_status h2_ctx_create(int device, void *stream, h2_ctx *out) {
  return guarded([&] {
    REQUIRE(out != nullptr, "null output");
    REQUIRE(device >= -1, "device must be >= -1");
    if (device >= 0) HIPCHK(hipSetDevice(device));
    auto c = std::make_unique<h2_ctx_s>();
    c->device = device;
    c->stream = (hipStream_t)stream;
    *out = c.release();
  });
}

h2_status h2_ctx_destroy(h2_ctx ctx) {
  delete ctx;
  return H2_OK;
}

h2_status h2_ctx_synchronize(h2_ctx ctx) {
  return guarded([&] {
    REQUIRE(ctx != nullptr, "null context");
    if (ctx->device >= 0) HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

static h2_status ctree_build(h2_ctx ctx, int32_t dim, int64_t n, const int32_t *coords,
                             int32_t leaf_size, bool dd, h2_ctree *out) {
  return guarded([&] {
    REQUIRE(ctx && coords && out, "null argument");
    REQUIRE(dim >= 1 && dim <= 3, "dim must be 1..3");
    REQUIRE(n >= 1 && n < (int64_t)1 << 30, "n out of range");
    REQUIRE(leaf_size >= 1 && leaf_size <= H2_MAX_LEAF, "leaf_size must be 1..H2_MAX_LEAF");
    auto ct = std::make_unique<h2_ctree_s>();
    ct->ctx = ctx; ct->n = n; ct->dim = dim; ct->leaf = leaf_size;
    build_ctree(*ct, coords, dd);
    *out = ct.release();
  });
}

h2_status h2_ctree_build(h2_ctx ctx, int32_t dim, int64_t n, const int32_t *coords, int32_t leaf_size,
                         h2_ctree *out) {
  return ctree_build(ctx, dim, n, coords, leaf_size, false, out);
}

h2_status h2_ctree_build_dd(h2_ctx ctx, int32_t dim, int64_t n, const int32_t *coords,
                            int32_t leaf_size, h2_ctree *out) {
  return ctree_build(ctx, dim, n, coords, leaf_size, true, out);
}

h2_status h2_ctree_info(h2_ctree ct, int64_t *n, int64_t *nclusters, int32_t *depth) {
  return guarded([&] {
    REQUIRE(ct != nullptr, "null tree");
    if (n) *n = ct->n;
    if (nclusters) *nclusters = ct->nc;
    if (depth) *depth = ct->depth;
  });
}

h2_status h2_ctree_export(h2_ctree ct, int64_t *perm, int32_t *offset, int32_t *size, int32_t *level,
                          int32_t *son0, int32_t *son1, int32_t *parent) {
  return guarded([&] {
    REQUIRE(ct != nullptr, "null tree");
    if (perm) std::copy(ct->perm.begin(), ct->perm.end(), perm);
    auto cp = [&](const std::vector<int> &v, int32_t *dst) { if (dst) std::copy(v.begin(), v.end(), dst); };
    cp(ct->offset, offset); cp(ct->size, size); cp(ct->level, level);
    cp(ct->son0, son0); cp(ct->son1, son1); cp(ct->parent, parent);
  });
}

h2_status h2_ctree_destroy(h2_ctree ct) {
  delete ct;
  return H2_OK;
}

h2_status h2_btree_build(h2_ctx ctx, h2_ctree ct, double eta, h2_btree *out) {
  return guarded([&] {
    REQUIRE(ctx && ct && out, "null argument");
    REQUIRE(eta > 0.0 && std::isfinite(eta), "eta must be positive");
    auto bt = std::make_unique<h2_btree_s>();
    bt->ctx = ctx; bt->ct = ct; bt->eta = eta;
    build_btree(*bt);
    *out = bt.release();
  });
}

h2_status h2_btree_info(h2_btree bt, int64_t *nblocks, int64_t *nadm, int64_t *nnear, int32_t *csp) {
  return guarded([&] {
    REQUIRE(bt != nullptr, "null tree");
    int64_t a = 0, nn = 0;
    std::vector<int> cnt(bt->ct->nc, 0);
    for (int b = 0; b < bt->nb; ++b) {
      if (bt->kind[b] == 1) { ++a; cnt[bt->row[b]]++; }
      if (bt->kind[b] == 2) ++nn;
    }
    if (nblocks) *nblocks = bt->nb;
    if (nadm) *nadm = a;
    if (nnear) *nnear = nn;
    if (csp) *csp = cnt.empty() ? 0 : *std::max_element(cnt.begin(), cnt.end());
  });
}

h2_status h2_btree_export(h2_btree bt, int32_t *row, int32_t *col, int32_t *kind, int32_t *parent) {
  return guarded([&] {
    REQUIRE(bt != nullptr, "null tree");
    auto cp = [&](const std::vector<int> &v, int32_t *dst) { if (dst) std::copy(v.begin(), v.end(), dst); };
    cp(bt->row, row); cp(bt->col, col); cp(bt->kind, kind); cp(bt->parent, parent);
  });
}

h2_status h2_btree_find(h2_btree bt, int64_t t, int64_t s, int64_t *block) {
  return guarded([&] {
    REQUIRE(bt && block, "null argument");
    REQUIRE(t >= 0 && s >= 0 && t < bt->ct->nc && s < bt->ct->nc, "cluster out of range");
    *block = bt->find((int)t, (int)s);
  });
}

h2_status h2_btree_destroy(h2_btree bt) {
  delete bt;
  return H2_OK;
}

h2_status h2_mat_from_csr(h2_ctx ctx, h2_btree bt, int64_t n, const int64_t *rowptr, const int32_t *col,
                          const double *val, int32_t lower, h2_mat *out) {
  return guarded([&] {
    REQUIRE(ctx && bt && rowptr && col && val && out, "null argument");
    const h2_ctree_s &ct = *bt->ct;
    REQUIRE(n == ct.n, "matrix size does not match the cluster tree");
    REQUIRE(ctx->device >= 0, "a host-only context cannot hold matrices");
    trees_to_device(*bt, ctx->stream);
    auto m = std::make_unique<h2_mat_s>();
    m->ctx = ctx; m->stream = ctx->stream; m->bt = bt; m->lower = lower != 0;
    mat_lists(*m);
    // cluster-order position and leaf of every index
    std::vector<int> pos(n), leafof(n);
    for (int64_t i = 0; i < n; ++i) pos[ct.perm[i]] = (int)i;
    for (int c = 0; c < ct.nc; ++c)
      if (ct.son0[c] < 0)
        for (int i = ct.offset[c]; i < ct.offset[c] + ct.size[c]; ++i) leafof[i] = c;
    std::vector<double> N((size_t)std::max(m->nnear, 1) * LS * LS, 0.0);
    for (int64_t i = 0; i < n; ++i) {
      for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        const double v = val[p];
        if (v == 0.0) continue;
        const int j = col[p];
        REQUIRE(j >= 0 && j < n, "column index out of range");
        const int ci = pos[i], cj = pos[j];
        const int t = leafof[ci], s = leafof[cj];
        const int b = bt->find(t, s);
        if (b < 0 || bt->kind[b] != 2)
          throw H2Error(H2_ERR_NONZERO_FARFIELD, "non-zero entry in an admissible block");
        const int slot = m->bslot[b];
        if (slot < 0) continue;   // upper triangle of a lower-stored matrix
        N[(size_t)slot * LS * LS + (ci - ct.offset[t]) + (size_t)(cj - ct.offset[s]) * LS] += v;
      }
    }
    mat_alloc(*m);
    hipStream_t s = ctx->stream;
    HIPCHK(hipMemcpyAsync(m->d_N.p, N.data(), N.size() * sizeof(double), hipMemcpyHostToDevice, s));
    mat_env(*m);
    HIPCHK(hipStreamSynchronize(s));
    *out = m.release();
  });
}

h2_status h2_mat_copy(h2_mat src, h2_mat *out) {
  return guarded([&] {
    REQUIRE(src && out, "null argument");
    require_ok(src);
    auto m = std::make_unique<h2_mat_s>();
    m->ctx = src->ctx; m->stream = src->stream; m->bt = src->bt; m->lower = src->lower;
    m->inverse = src->inverse;
    std::copy(src->prec_nt, src->prec_nt + BC + 1, m->prec_nt);
    mat_lists(*m);
    mat_alloc(*m);
    hipStream_t s = src->ctx->stream;
    auto cp = [&](auto &dst, auto &from) {
      if (from.n) HIPCHK(hipMemcpyAsync(dst.p, from.p, from.n * sizeof(*from.p), hipMemcpyDeviceToDevice, s));
    };
    for (int side = 0; side < 2; ++side) {
      cp(m->d_k[side], src->d_k[side]); cp(m->d_rho_m[side], src->d_rho_m[side]);
      cp(m->d_leaf[side], src->d_leaf[side]); cp(m->d_E[side], src->d_E[side]);
      cp(m->d_rho[side], src->d_rho[side]);
    }
    cp(m->d_S, src->d_S); cp(m->d_N, src->d_N);
    mat_env(*m);
    HIPCHK(hipStreamSynchronize(s));
    *out = m.release();
  });
}

h2_status h2_mat_assign(h2_mat dst, h2_mat src) {
  return guarded([&] {
    REQUIRE(dst && src, "null argument");
    require_ok(src);
    REQUIRE(!dst->busy, "matrix belongs to an unfinished batch (finish its job first)");
    REQUIRE(dst->bt == src->bt && dst->lower == src->lower, "matrices have different structure");
    hipStream_t s = dst->ctx->stream;
    auto cp = [&](auto &to, auto &from) {
      if (from.n) HIPCHK(hipMemcpyAsync(to.p, from.p, from.n * sizeof(*from.p), hipMemcpyDeviceToDevice, s));
    };
    for (int side = 0; side < 2; ++side) {
      cp(dst->d_k[side], src->d_k[side]); cp(dst->d_rho_m[side], src->d_rho_m[side]);
      cp(dst->d_leaf[side], src->d_leaf[side]); cp(dst->d_E[side], src->d_E[side]);
      cp(dst->d_rho[side], src->d_rho[side]);
    }
    cp(dst->d_S, src->d_S); cp(dst->d_N, src->d_N);
    HIPCHK(hipMemsetAsync(dst->d_err.p, 0, dst->d_err.n * sizeof(int), s));
    dst->poisoned = false;
    dst->inverse = src->inverse;
    dst->lr = src->lr;
  });
}

h2_status h2_mat_flops(h2_mat m, double *flops, int32_t reset) {
  return guarded([&] {
    REQUIRE(m != nullptr, "null matrix");
    hipStream_t s = m->ctx->stream;
    if (flops) {
      std::vector<double> h(m->d_flops.n);
      HIPCHK(hipMemcpyAsync(h.data(), m->d_flops.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      double sum = 0.0;
      for (double v : h) sum += v;
      *flops = sum;
    }
    if (reset) m->d_flops.zero(s);
  });
}

h2_status h2_profile(h2_mat m, int32_t enable, int64_t *counters, int32_t n) {
  return guarded([&] {
    REQUIRE(m != nullptr, "null matrix");
    hipStream_t s = m->ctx->stream;
    if (counters && m->d_prof.p) {
      REQUIRE(n >= 0 && n <= PROF_LEN, "too many counters");
      std::vector<unsigned long long> h(PROF_LEN);
      HIPCHK(hipMemcpyAsync(h.data(), m->d_prof.p, PROF_LEN * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int i = 0; i < n; ++i) counters[i] = (int64_t)h[i];
    }
    if (enable) {
      if (!m->d_prof.p) m->d_prof.alloc_on(PROF_LEN, m->stream);
      m->d_prof.zero(s);
      m->env.prof = m->d_prof.p;
    } else {
      m->env.prof = nullptr;
    }
  });
}

h2_status h2_mat_destroy(h2_mat m) {
  // Touches no other object: handles may be destroyed in any order.
  if (m && m->busy) {
    g_last_error = "matrix belongs to an unfinished batch (finish its job first)";
    return H2_ERR_STATE;
  }
  if (m) (void)hipStreamSynchronize(m->stream);
  delete m;
  return H2_OK;
}

h2_status h2_estimate_bytes(h2_btree bt, int32_t lower, int64_t *bytes) {
  return guarded([&] {
    REQUIRE(bt != nullptr && bytes != nullptr, "null argument");
    *bytes = (int64_t)mat_bytes_planned(*bt, lower != 0);
  });
}

h2_status h2_mat_bytes(h2_mat m, int64_t *bytes) {
  return guarded([&] {
    REQUIRE(m != nullptr && bytes != nullptr, "null argument");
    *bytes = (int64_t)mat_bytes_now(*m);
  });
}

h2_status h2_mat_ranks(h2_mat m, int32_t *rank_row, int32_t *rank_col) {
  return guarded([&] {
    REQUIRE(m != nullptr, "null matrix");
    const int nc = (int)m->bt->ct->nc;
    int32_t *dst[2] = {rank_row, rank_col};
    for (int side = 0; side < 2; ++side)
      if (dst[side])
        HIPCHK(hipMemcpyAsync(dst[side], m->d_k[side].p, nc * sizeof(int), hipMemcpyDeviceToHost, m->ctx->stream));
    HIPCHK(hipStreamSynchronize(m->ctx->stream));
  });
}

h2_status h2_mat_stats(h2_mat m, int64_t *stored_values, int32_t *max_rank_row, int32_t *max_rank_col) {
  return guarded([&] {
    REQUIRE(m != nullptr, "null matrix");
    int kr = 0, kc = 0;
    const int64_t vals = mat_stored_values(*m, &kr, &kc);
    if (stored_values) *stored_values = vals;
    if (max_rank_row) *max_rank_row = kr;
    if (max_rank_col) *max_rank_col = kc;
  });
}

h2_status h2_lowrank_update(h2_mat z, int64_t block, int32_t k, const double *X, int64_t ldx,
                            const double *Y, int64_t ldy, const h2_trunc *tr) {
  return guarded([&] {
    require_ok(z);
    require_validated_tree(*z);
    const h2_btree_s &bt = *z->bt;
    const h2_ctree_s &ct = *bt.ct;
    REQUIRE(block >= 0 && block < bt.nb, "block out of range");
    REQUIRE(k >= 0 && k <= H2_MAX_UPDATE_RANK, "update rank out of range");
    const int t0 = bt.row[block], s0 = bt.col[block];
    if (z->lower) REQUIRE(t0 == s0 || ct.offset[t0] > ct.offset[s0], "block above the diagonal of a lower matrix");
    if (k == 0) return;
    REQUIRE(X && Y, "null factor");
    REQUIRE(ldx >= ct.size[t0] && ldy >= ct.size[s0], "leading dimension too small");
    set_trunc(*z, tr);
    hipStream_t s = z->ctx->stream;
    hipLaunchKernelGGL(k_gather, dim3(grid_for((long)ct.size[t0] * k)), dim3(256), 0, s, ct.size[t0],
                       ct.offset[t0], k, (const int64_t *)nullptr, X, (long)ldx, z->env.buf[B_X], z->d_bcols.p,
                       (int)B_X);
    hipLaunchKernelGGL(k_gather, dim3(grid_for((long)ct.size[s0] * k)), dim3(256), 0, s, ct.size[s0],
                       ct.offset[s0], k, (const int64_t *)nullptr, Y, (long)ldy, z->env.buf[B_Y], z->d_bcols.p,
                       (int)B_Y);
    HIPCHK(hipGetLastError());
    std::vector<Task> tasks;
    Planner P(*z, tasks);
    P.addlr((int)block, B_X, B_Y);
    TaskList tl;
    upload_tasks(*z, tl, tasks, P.aux);
    run_tasks(*z, tl);
    check_device_error(*z);
  });
}

// Smallest block of the block tree containing every block in the list: the
// deepest common ancestor (the ancestors of a block are the blocks that
// contain it).
static int common_block(const h2_btree_s &bt, const int64_t *blocks, int count) {
  std::vector<int> path;   // ancestors of the first block, deepest first
  for (int b = (int)blocks[0]; b >= 0; b = bt.parent[b]) path.push_back(b);
  std::vector<char> keep(path.size(), 1);
  for (int i = 1; i < count; ++i) {
    std::vector<char> seen(path.size(), 0);
    for (int b = (int)blocks[i]; b >= 0; b = bt.parent[b])
      for (size_t j = 0; j < path.size(); ++j)
        if (path[j] == b) seen[j] = 1;
    for (size_t j = 0; j < path.size(); ++j) keep[j] = keep[j] && seen[j];
  }
  for (size_t j = 0; j < path.size(); ++j)
    if (keep[j]) return path[j];
  return 0;   // the root contains every block
}

h2_status h2_lowrank_update_accumulated(h2_mat z, int32_t count, const int64_t *blocks, const int32_t *ks,
                                        const double *const *Xs, const int64_t *ldxs, const double *const *Ys,
                                        const int64_t *ldys, const h2_trunc *tr, int64_t *merged_block) {
  return guarded([&] {
    require_ok(z);
    require_validated_tree(*z);
    REQUIRE(count >= 1 && blocks && ks && Xs && ldxs && Ys && ldys, "null argument or empty list");
    const h2_btree_s &bt = *z->bt;
    const h2_ctree_s &ct = *bt.ct;
    int ktot = 0;
    for (int i = 0; i < count; ++i) {
      REQUIRE(blocks[i] >= 0 && blocks[i] < bt.nb, "block out of range");
      REQUIRE(ks[i] >= 0 && ks[i] <= H2_MAX_UPDATE_RANK, "update rank out of range");
      const int t = bt.row[blocks[i]], c = bt.col[blocks[i]];
      if (z->lower) REQUIRE(t == c || ct.offset[t] > ct.offset[c], "block above the diagonal of a lower matrix");
      if (ks[i] == 0) continue;
      REQUIRE(Xs[i] && Ys[i], "null factor");
      REQUIRE(ldxs[i] >= ct.size[t] && ldys[i] >= ct.size[c], "leading dimension too small");
      ktot += ks[i];
    }
    REQUIRE(ktot <= H2_MAX_UPDATE_RANK, "accumulated rank above H2_MAX_UPDATE_RANK");
    const int bs = common_block(bt, blocks, count);
    const int ts = bt.row[bs], ss = bt.col[bs];
    if (z->lower) REQUIRE(ts == ss || ct.offset[ts] > ct.offset[ss], "internal: merged block above the diagonal");
    if (merged_block) *merged_block = bs;
    if (ktot == 0) return;
    set_trunc(*z, tr);
    hipStream_t s = z->ctx->stream;
    // merged factors: the rows of t* (s*) in the update buffers, cleared,
    // then every factor at its rows and its own columns
    const int side_rows[2] = {ts, ss};
    const int bufs[2] = {B_X, B_Y};
    for (int side = 0; side < 2; ++side) {
      const int c = side_rows[side];
      const long len = (long)ct.size[c] * BC;
      hipLaunchKernelGGL(k_fill_double, dim3(grid_for(len)), dim3(256), 0, s,
                         z->env.buf[bufs[side]] + (long)ct.offset[c] * BC, (int)len, 0.0);
    }
    int col0 = 0;
    for (int i = 0; i < count; ++i) {
      const int k = ks[i];
      if (k == 0) continue;
      const int t = bt.row[blocks[i]], c = bt.col[blocks[i]];
      hipLaunchKernelGGL(k_gather, dim3(grid_for((long)ct.size[t] * k)), dim3(256), 0, s, ct.size[t],
                         ct.offset[t], k, (const int64_t *)nullptr, Xs[i], (long)ldxs[i],
                         z->env.buf[B_X] + col0, z->d_bcols.p, (int)B_X);
      hipLaunchKernelGGL(k_gather, dim3(grid_for((long)ct.size[c] * k)), dim3(256), 0, s, ct.size[c],
                         ct.offset[c], k, (const int64_t *)nullptr, Ys[i], (long)ldys[i],
                         z->env.buf[B_Y] + col0, z->d_bcols.p, (int)B_Y);
      col0 += k;
    }
    for (int side = 0; side < 2; ++side)
      hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, z->d_bcols.p + bufs[side], 1, ktot);
    HIPCHK(hipGetLastError());
    std::vector<Task> tasks;
    Planner P(*z, tasks);
    P.addlr(bs, B_X, B_Y);
    TaskList tl;
    upload_tasks(*z, tl, tasks, P.aux);
    run_tasks(*z, tl);
    check_device_error(*z);
  });
}

h2_status h2_matvec(h2_mat z, int32_t trans, double alpha, const double *x, double beta, double *y,
                    int32_t nrhs) {
  return guarded([&] {
    require_ok(z);
    REQUIRE(x && y, "null vector");
    REQUIRE(nrhs >= 1 && nrhs <= H2_MAX_COLS, "nrhs out of range");
    const h2_ctree_s &ct = *z->bt->ct;
    hipStream_t s = z->ctx->stream;
    const long work = (long)ct.n * nrhs;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(work)), dim3(256), 0, s, (int)ct.n, 0, nrhs, ct.d_perm.p, x,
                       (long)ct.n, z->env.buf[B_X], z->d_bcols.p, (int)B_X);
    HIPCHK(hipGetLastError());
    std::vector<Task> tasks;
    Planner P(*z, tasks);
    P.bapply(0, trans ? 1 : 0, B_X, B_Y, 1.0, 0.0);
    TaskList tl;
    upload_tasks(*z, tl, tasks, P.aux);
    run_tasks(*z, tl);
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(work)), dim3(256), 0, s, (int)ct.n, nrhs, ct.d_perm.p,
                       z->env.buf[B_Y], y, (long)ct.n, alpha, beta);
    HIPCHK(hipGetLastError());
    check_device_error(*z);
  });
}

h2_status h2_cholesky(h2_mat a, const h2_trunc *tr) {
  return guarded([&] {
    require_ok(a);
    REQUIRE(a->lower, "h2_cholesky needs a matrix created with lower != 0");
    require_validated_tree(*a);
    REQUIRE(!a->inverse, "h2_cholesky on an inverted factor");
    set_trunc(*a, tr);
    if (!a->chol.built) {
      std::vector<Task> tasks;
      Planner P(*a, tasks);
      P.chol(0);
      upload_tasks(*a, a->chol, tasks, P.aux);
    }
    run_tasks(*a, a->chol);
    check_device_error(*a);
  });
}

h2_status h2_lr(h2_mat a, const h2_trunc *tr) {
  return guarded([&] {
    require_ok(a);
    REQUIRE(!a->lower, "h2_lr needs a matrix created with lower = 0 (full storage)");
    require_validated_tree(*a);
    set_trunc(*a, tr);
    if (!a->lrf.built) {
      std::vector<Task> tasks;
      Planner P(*a, tasks);
      P.lr(0);
      upload_tasks(*a, a->lrf, tasks, P.aux);
    }
    a->lr = false;
    run_tasks(*a, a->lrf);
    check_device_error(*a);
    a->lr = true;
  });
}

// Environment through which the product's tasks read the operand m: m's
// matrix data with the target z's work areas, error flag, counters and
// truncation parameters.
static DevEnv operand_env(const h2_mat_s &m, const h2_mat_s &z) {
  DevEnv e = m.env;
  const DevEnv &t = z.env;
  e.rank_cap = t.rank_cap; e.mode = t.mode; e.eps = t.eps; e.prec = t.prec;
  for (int side = 0; side < 2; ++side) {
    e.wrho[side] = t.wrho[side]; e.wrho_m[side] = t.wrho_m[side];
    e.wB[side] = t.wB[side]; e.wB_m[side] = t.wB_m[side];
    e.wR[side] = t.wR[side]; e.wnewk[side] = t.wnewk[side];
  }
  e.xh = t.xh; e.yh = t.yh;
  for (int i = 0; i < NBUF; ++i) e.buf[i] = t.buf[i];
  e.bcols = t.bcols; e.err = t.err; e.prof = t.prof; e.flops = t.flops; e.wscr = t.wscr;
  return e;
}

h2_status h2_product(h2_mat z, double alpha, h2_mat x, h2_mat y, const h2_trunc *tr) {
  return guarded([&] {
    require_ok(z); require_ok(x); require_ok(y);
    REQUIRE(z != x && z != y, "h2_product: the target must differ from both factors");
    require_validated_tree(*z);
    REQUIRE(!z->lower && !x->lower && !y->lower, "h2_product needs full-storage matrices (lower = 0)");
    REQUIRE(x->bt == z->bt && y->bt == z->bt, "h2_product: the matrices must share one block tree");
    REQUIRE(x->ctx->device == z->ctx->device && y->ctx->device == z->ctx->device,
            "h2_product: the matrices must live on one device");
    // the factors are read on z's stream: finish their own pending work
    for (h2_mat m : {x, y})
      if (m->stream != z->stream) HIPCHK(hipStreamSynchronize(m->stream));
    set_trunc(*z, tr);
    if (!z->prod.built || z->prod_alpha != alpha) {
      // alpha is stored in the emitted tasks: planned again for another value
      std::vector<Task> tasks;
      Planner P(*z, tasks);
      P.ex = 1;
      P.ey = 2;
      P.mm_n(0, 0, 0, alpha, -1, 0, 0);
      upload_tasks(*z, z->prod, tasks, P.aux);
      z->prod_alpha = alpha;
    }
    const DevEnv envs[3] = {z->env, operand_env(*x, *z), operand_env(*y, *z)};
    if (!z->d_env3.p) z->d_env3.alloc_on(3, z->stream);
    HIPCHK(hipMemcpyAsync(z->d_env3.p, envs, sizeof envs, hipMemcpyHostToDevice, z->stream));
    HIPCHK(hipStreamSynchronize(z->stream));
    run_tasks(*z, z->prod, NT, z->d_env3.p);
    check_device_error(*z);
  });
}

static bool g_lds_attr_batch_set = false;

// Device arrays of batch descriptors are recycled, never freed: freeing
// device memory waits for the whole device, which would stall the host
// while launches on other streams run.
static std::mutex g_items_mu;
static std::vector<Dev<BatchItem> *> g_items_free;

static Dev<BatchItem> *items_acquire(size_t count) {
  std::lock_guard<std::mutex> lk(g_items_mu);
  for (size_t i = 0; i < g_items_free.size(); ++i)
    if (g_items_free[i]->n >= count) {
      Dev<BatchItem> *d = g_items_free[i];
      g_items_free.erase(g_items_free.begin() + i);
      return d;
    }
  auto *d = new Dev<BatchItem>();
  try {
    d->alloc(std::max<size_t>(count, 64));
  } catch (...) {
    d->p = nullptr;   // nothing to free
    delete d;
    throw;
  }
  return d;
}

static void items_release(Dev<BatchItem> *d) {
  if (!d) return;
  std::lock_guard<std::mutex> lk(g_items_mu);
  g_items_free.push_back(d);
}

// One k_interp_batch launch over items (uploaded from the host vector, which
// must stay untouched until the stream has passed the launch).
static void launch_batch(Dev<BatchItem> &d_items, const std::vector<BatchItem> &items, int nthreads,
                         hipStream_t s) {
  const size_t lds = LDS_TOTAL_DOUBLES * sizeof(double);
  if (!g_lds_attr_batch_set) {
    HIPCHK(hipFuncSetAttribute((const void *)k_interp_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    g_lds_attr_batch_set = true;
  }
  REQUIRE(d_items.n >= items.size(), "internal: descriptor array too small");
  HIPCHK(hipMemcpyAsync(d_items.p, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_interp_batch, dim3((unsigned)items.size()), dim3(nthreads), lds, s,
                     (const BatchItem *)d_items.p);
  HIPCHK(hipGetLastError());
}

// Checks of a batch: distinct matrices, usable, on one device and stream.
static std::vector<h2_mat_s *> batch_members(h2_mat *mats, int32_t count, const char *what,
                                             bool factors = true) {
  REQUIRE(mats != nullptr && count >= 1, "need at least one matrix");
  std::vector<h2_mat_s *> ms(mats, mats + count);
  for (h2_mat_s *m : ms) {
    require_ok(m);
    if (factors) {
      REQUIRE(m->lower, (std::string(what) + " needs matrices created with lower != 0").c_str());
      REQUIRE(!m->inverse, (std::string(what) + " on an inverted factor").c_str());
    }
    REQUIRE(m->ctx->device == ms[0]->ctx->device && m->ctx->stream == ms[0]->ctx->stream,
            "all matrices of a batch must share one device and stream");
  }
  std::vector<h2_mat_s *> sorted(ms);
  std::sort(sorted.begin(), sorted.end());
  REQUIRE(std::adjacent_find(sorted.begin(), sorted.end()) == sorted.end(), "a matrix appears twice in the batch");
  return ms;
}

// Checks every matrix of a finished batch; failed ones are poisoned and
// their status stored, the first failure is rethrown.
static void batch_errors(const std::vector<h2_mat_s *> &ms, h2_status *status) {
  bool failed = false;
  H2Error first(H2_OK, "");
  for (size_t i = 0; i < ms.size(); ++i) {
    try {
      check_device_error(*ms[i]);
    } catch (const H2Error &e) {
      if (status) status[i] = e.code;
      if (!failed) {
        first = H2Error(e.code, "matrix " + std::to_string(i) + " of the batch: " + e.what());
        failed = true;
      }
    }
  }
  if (failed) throw first;
}

}  // extern "C"

// Argument checks of a batch of local updates (before any device work):
// matrix i receives nupd[i] updates from the flat arrays.
static void check_update_batch(const std::vector<h2_mat_s *> &ms, const int32_t *nupd, const int64_t *blocks,
                               const int32_t *ks, const double *const *Xs, const int64_t *ldxs,
                               const double *const *Ys, const int64_t *ldys) {
  int u0 = 0;
  for (size_t i = 0; i < ms.size(); ++i) {
    const h2_mat_s &z = *ms[i];
    const h2_btree_s &bt = *z.bt;
    const h2_ctree_s &ct = *bt.ct;
    REQUIRE(nupd[i] >= 0 && nupd[i] <= H2_MAX_BATCH_UPDATES, "updates per matrix out of range");
    for (int u = u0; u < u0 + nupd[i]; ++u) {
      REQUIRE(blocks[u] >= 0 && blocks[u] < bt.nb, "block out of range");
      REQUIRE(ks[u] >= 0 && ks[u] <= H2_MAX_UPDATE_RANK, "update rank out of range");
      const int t0 = bt.row[blocks[u]], s0 = bt.col[blocks[u]];
      if (z.lower) REQUIRE(t0 == s0 || ct.offset[t0] > ct.offset[s0], "block above the diagonal of a lower matrix");
      if (ks[u] == 0) continue;
      REQUIRE(Xs[u] && Ys[u], "null factor");
      REQUIRE(ldxs[u] >= ct.size[t0] && ldys[u] >= ct.size[s0], "leading dimension too small");
    }
    u0 += nupd[i];
  }
}

// Plans the updates of every matrix of a checked batch into its own task
// list and gathers the factors on the batch's stream; returns one launch
// descriptor per matrix.  Update j's factors go to the j-th pair of product
// temporaries, which the local update itself leaves untouched; a matrix's
// updates run in order.
static std::vector<BatchItem> plan_update_batch(const std::vector<h2_mat_s *> &ms, const int32_t *nupd,
                                                const int64_t *blocks, const int32_t *ks,
                                                const double *const *Xs, const int64_t *ldxs,
                                                const double *const *Ys, const int64_t *ldys,
                                                const h2_trunc *tr) {
  hipStream_t s = ms[0]->ctx->stream;
  std::vector<BatchItem> items(ms.size());
  int u0 = 0;
  for (size_t i = 0; i < ms.size(); ++i) {
    h2_mat_s &z = *ms[i];
    const h2_btree_s &bt = *z.bt;
    const h2_ctree_s &ct = *bt.ct;
    set_trunc(z, tr);
    std::vector<Task> tasks;
    Planner P(z, tasks);
    for (int j = 0; j < nupd[i]; ++j) {
      const int u = u0 + j, k = ks[u];
      if (k == 0) continue;
      const int b = (int)blocks[u], t0 = bt.row[b], s0 = bt.col[b];
      const int bu = B_T0U + 2 * j, bv = B_T0V + 2 * j;
      hipLaunchKernelGGL(k_gather, dim3(grid_for((long)ct.size[t0] * k)), dim3(256), 0, s, ct.size[t0],
                         ct.offset[t0], k, (const int64_t *)nullptr, Xs[u], (long)ldxs[u], z.env.buf[bu],
                         z.d_bcols.p, bu);
      hipLaunchKernelGGL(k_gather, dim3(grid_for((long)ct.size[s0] * k)), dim3(256), 0, s, ct.size[s0],
                         ct.offset[s0], k, (const int64_t *)nullptr, Ys[u], (long)ldys[u], z.env.buf[bv],
                         z.d_bcols.p, bv);
      HIPCHK(hipGetLastError());
      P.addlr(b, bu, bv);
    }
    upload_tasks_reuse(z.upd, tasks, P.aux);
    sync_env(z);
    items[i] = BatchItem{z.upd.d.p, z.d_env.p, z.upd.aux.p, z.upd.count, 0};
    u0 += nupd[i];
  }
  return items;
}

// Plans (first call per matrix) the Cholesky factorisation of every matrix
// of a batch; returns one launch descriptor per matrix.
static std::vector<BatchItem> plan_cholesky_batch(const std::vector<h2_mat_s *> &ms, const h2_trunc *tr) {
  std::vector<BatchItem> items(ms.size());
  for (size_t i = 0; i < ms.size(); ++i) {
    h2_mat_s &m = *ms[i];
    set_trunc(m, tr);
    if (!m.chol.built) {
      std::vector<Task> tasks;
      Planner P(m, tasks);
      P.chol(0);
      upload_tasks(m, m.chol, tasks, P.aux);
    }
    sync_env(m);
    items[i] = BatchItem{m.chol.d.p, m.d_env.p, m.chol.aux.p, m.chol.count, 0};
  }
  return items;
}

struct h2_job_s {
  std::vector<h2_mat_s *> ms;
  std::vector<BatchItem> items;
  Dev<BatchItem> *d_items = nullptr;
  hipEvent_t done = nullptr;
  hipStream_t stream = nullptr;
  ~h2_job_s() {
    if (done) {
      (void)hipEventSynchronize(done);
      (void)hipEventDestroy(done);
    } else if (d_items) {
      (void)hipStreamSynchronize(stream);   // launched but no event: wait before reuse
    }
    items_release(d_items);
    for (h2_mat_s *m : ms) m->busy = false;
  }
};

// One launch of k_interp_batch over the local updates of the matrices us
// (a matrix's updates in order) and the Cholesky factorisations of the
// matrices cs, one workgroup each.
static void update_cholesky_launch(h2_mat *umats, int32_t ucount, const int32_t *nupd, const int64_t *blocks,
                                   const int32_t *ks, const double *const *Xs, const int64_t *ldxs,
                                   const double *const *Ys, const int64_t *ldys, h2_mat *cmats, int32_t ccount,
                                   const h2_trunc *tr, h2_job *job, const char *what) {
  REQUIRE(job != nullptr, "null output");
  *job = nullptr;
  REQUIRE(ucount >= 0 && ccount >= 0 && ucount + ccount >= 1, "need at least one matrix");
  std::vector<h2_mat_s *> us, cs;
  if (ucount > 0) {
    REQUIRE(nupd && blocks && ks && Xs && ldxs && Ys && ldys, "null argument");
    us = batch_members(umats, ucount, what, false);
  }
  if (ccount > 0) cs = batch_members(cmats, ccount, what);
  std::vector<h2_mat_s *> all(us);
  all.insert(all.end(), cs.begin(), cs.end());
  for (h2_mat_s *m : all) {
    REQUIRE(m->ctx->device == all[0]->ctx->device && m->ctx->stream == all[0]->ctx->stream,
            "all matrices of a batch must share one device and stream");
    require_validated_tree(*m);
  }
  {
    std::vector<h2_mat_s *> sorted(all);
    std::sort(sorted.begin(), sorted.end());
    REQUIRE(std::adjacent_find(sorted.begin(), sorted.end()) == sorted.end(),
            "a matrix appears twice in the batch");
  }
  if (ucount > 0) check_update_batch(us, nupd, blocks, ks, Xs, ldxs, Ys, ldys);
  auto j = std::make_unique<h2_job_s>();
  if (ucount > 0) j->items = plan_update_batch(us, nupd, blocks, ks, Xs, ldxs, Ys, ldys, tr);
  if (ccount > 0) {
    const std::vector<BatchItem> ci = plan_cholesky_batch(cs, tr);
    j->items.insert(j->items.end(), ci.begin(), ci.end());
  }
  j->stream = all[0]->ctx->stream;
  j->d_items = items_acquire(j->items.size());
  launch_batch(*j->d_items, j->items, NT, j->stream);
  HIPCHK(hipEventCreateWithFlags(&j->done, hipEventDisableTiming));
  HIPCHK(hipEventRecord(j->done, j->stream));
  j->ms = all;
  for (h2_mat_s *m : all) m->busy = true;
  *job = j.release();
}

extern "C" {

h2_status h2_cholesky_launch(h2_mat *mats, int32_t count, const h2_trunc *tr, h2_job *job) {
  return guarded([&] {
    REQUIRE(mats != nullptr && count >= 1, "need at least one matrix");
    update_cholesky_launch(nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, mats, count,
                           tr, job, "h2_cholesky_launch");
  });
}

h2_status h2_update_cholesky_launch(h2_mat *umats, int32_t ucount, const int32_t *nupd, const int64_t *blocks,
                                    const int32_t *ks, const double *const *Xs, const int64_t *ldxs,
                                    const double *const *Ys, const int64_t *ldys, h2_mat *cmats,
                                    int32_t ccount, const h2_trunc *tr, h2_job *job) {
  return guarded([&] {
    update_cholesky_launch(umats, ucount, nupd, blocks, ks, Xs, ldxs, Ys, ldys, cmats, ccount, tr, job,
                           "h2_update_cholesky_launch");
  });
}

h2_status h2_job_query(h2_job job, int32_t *done) {
  return guarded([&] {
    REQUIRE(job != nullptr && done != nullptr, "null argument");
    const hipError_t e = hipEventQuery(job->done);
    if (e == hipErrorNotReady) { *done = 0; return; }
    HIPCHK(e);
    *done = 1;
  });
}

h2_status h2_job_finish(h2_job job, h2_status *status) {
  return guarded([&] {
    REQUIRE(job != nullptr, "null job");
    std::unique_ptr<h2_job_s> j(job);
    if (status)
      for (size_t i = 0; i < j->ms.size(); ++i) status[i] = H2_OK;
    HIPCHK(hipEventSynchronize(j->done));
    for (h2_mat_s *m : j->ms) m->busy = false;
    batch_errors(j->ms, status);
  });
}

h2_status h2_lowrank_update_batched(h2_mat *mats, int32_t count, const int32_t *nupd, const int64_t *blocks,
                                   const int32_t *ks, const double *const *Xs, const int64_t *ldxs,
                                   const double *const *Ys, const int64_t *ldys, const h2_trunc *tr,
                                   h2_status *status) {
  return guarded([&] {
    REQUIRE(nupd && blocks && ks && Xs && ldxs && Ys && ldys, "null argument");
    std::vector<h2_mat_s *> ms = batch_members(mats, count, "h2_lowrank_update_batched", false);
    for (h2_mat_s *m : ms) require_validated_tree(*m);
    if (status)
      for (int i = 0; i < count; ++i) status[i] = H2_OK;
    check_update_batch(ms, nupd, blocks, ks, Xs, ldxs, Ys, ldys);
    hipStream_t s = ms[0]->ctx->stream;
    const std::vector<BatchItem> items = plan_update_batch(ms, nupd, blocks, ks, Xs, ldxs, Ys, ldys, tr);
    struct ItemsGuard {
      Dev<BatchItem> *d; hipStream_t s;
      ~ItemsGuard() { (void)hipStreamSynchronize(s); items_release(d); }
    } guard{items_acquire(count), s};
    launch_batch(*guard.d, items, NT, s);
    HIPCHK(hipStreamSynchronize(s));
    batch_errors(ms, status);
  });
}

h2_status h2_cholesky_batched(h2_mat *mats, int32_t count, const h2_trunc *tr, h2_status *status) {
  h2_job job = nullptr;
  const h2_status st = h2_cholesky_launch(mats, count, tr, &job);
  if (st != H2_OK) return st;
  return h2_job_finish(job, status);
}

// z = G^* G r for an inverted factor G ~ L^{-1}: two products with the
// lower triangular H^2 matrix (all stored leaves, every level at once).
static void precond_inverse_device(h2_mat g, const double *r, double *z, int nrhs) {
  const h2_ctree_s &ct = *g->bt->ct;
  hipStream_t s = g->ctx->stream;
  if (!g->prec_inv.built) {
    std::vector<Task> tasks;
    Planner P(*g, tasks);
    P.bapply(0, 0, B_X, B_Y, 1.0, 0.0);
    P.bapply(0, 1, B_Y, B_X, 1.0, 0.0);
    upload_tasks(*g, g->prec_inv, tasks, P.aux);
  }
  const long work = (long)ct.n * nrhs;
  hipLaunchKernelGGL(k_gather, dim3(grid_for(work)), dim3(256), 0, s, (int)ct.n, 0, nrhs, ct.d_perm.p, r,
                     (long)ct.n, g->env.buf[B_X], g->d_bcols.p, (int)B_X);
  HIPCHK(hipGetLastError());
  run_tasks(*g, g->prec_inv);
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(work)), dim3(256), 0, s, (int)ct.n, nrhs, ct.d_perm.p,
                     g->env.buf[B_X], z, (long)ct.n, 1.0, 0.0);
  HIPCHK(hipGetLastError());
}

// Task list of the forward and backward substitution with a factor L.
static const TaskList &prec_list(h2_mat l) {
  if (!l->prec.built) {
    std::vector<Task> tasks;
    Planner P(*l, tasks);
    P.fsolve_h2(0, B_X);
    P.bsolve_h2(0, B_X);
    upload_tasks(*l, l->prec, tasks, P.aux);
  }
  return l->prec;
}

// The substitution tasks (and the leaf solves) use the run-time wave count
// (at least two waves: the push to the sons takes one wave per son); every
// column, cluster and block group is computed by one wave in a fixed order,
// so the result does not depend on the count.  Default four waves;
// h2_autotune_precond picks per matrix and column count.
constexpr int PREC_THREADS = 256;
constexpr int PREC_SHAPES[3] = {128, 256, 512};

static int prec_threads(const h2_mat_s &l, int nrhs) {
  const int t = (nrhs >= 1 && nrhs <= BC) ? l.prec_nt[nrhs] : 0;
  return t > 0 ? t : PREC_THREADS;
}

static void prec_gather(h2_mat l, const double *r, int nrhs) {
  const h2_ctree_s &ct = *l->bt->ct;
  const long work = (long)ct.n * nrhs;
  hipLaunchKernelGGL(k_gather, dim3(grid_for(work)), dim3(256), 0, l->ctx->stream, (int)ct.n, 0, nrhs,
                     ct.d_perm.p, r, (long)ct.n, l->env.buf[B_X], l->d_bcols.p, (int)B_X);
  HIPCHK(hipGetLastError());
}

static void prec_scatter(h2_mat l, double *z, int nrhs) {
  const h2_ctree_s &ct = *l->bt->ct;
  const long work = (long)ct.n * nrhs;
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(work)), dim3(256), 0, l->ctx->stream, (int)ct.n, nrhs,
                     ct.d_perm.p, l->env.buf[B_X], z, (long)ct.n, 1.0, 0.0);
  HIPCHK(hipGetLastError());
}

static void precond_device(h2_mat l, const double *r, double *z, int nrhs) {
  if (l->inverse) { precond_inverse_device(l, r, z, nrhs); return; }
  const TaskList &tl = prec_list(l);
  prec_gather(l, r, nrhs);
  run_tasks(*l, tl, prec_threads(*l, nrhs));
  prec_scatter(l, z, nrhs);
}

h2_status h2_tri_invert(h2_mat l, const h2_trunc *tr) {
  return guarded([&] {
    require_ok(l);
    REQUIRE(l->lower, "h2_tri_invert needs a lower triangular factor");
    require_validated_tree(*l);
    REQUIRE(!l->inverse, "matrix is already inverted");
    set_trunc(*l, tr);
    if (!l->tinv.built) {
      std::vector<Task> tasks;
      Planner P(*l, tasks);
      P.tinv(0);
      upload_tasks(*l, l->tinv, tasks, P.aux);
    }
    run_tasks(*l, l->tinv);
    l->inverse = true;
    check_device_error(*l);
  });
}

h2_status h2_mat_is_inverse(h2_mat m, int32_t *inverse) {
  return guarded([&] {
    REQUIRE(m && inverse, "null argument");
    *inverse = m->inverse ? 1 : 0;
  });
}

h2_status h2_precond(h2_mat l, const double *r, double *z, int32_t nrhs) {
  return guarded([&] {
    require_ok(l);
    REQUIRE(l->lower, "h2_precond needs a Cholesky factor");
    REQUIRE(r && z, "null vector");
    REQUIRE(nrhs >= 1 && nrhs <= H2_MAX_COLS, "nrhs out of range");
    precond_device(l, r, z, nrhs);
    check_device_error(*l);
  });
}

h2_status h2_trsv(h2_mat l, int32_t trans, const double *r, double *z, int32_t nrhs) {
  return guarded([&] {
    require_ok(l);
    REQUIRE(l->lower, "h2_trsv needs a Cholesky factor");
    REQUIRE(!l->inverse, "h2_trsv on an inverted factor");
    REQUIRE(trans == 0 || trans == 1, "trans must be 0 or 1");
    REQUIRE(r && z, "null vector");
    REQUIRE(nrhs >= 1 && nrhs <= H2_MAX_COLS, "nrhs out of range");
    TaskList &tl = l->trsv[trans];
    if (!tl.built) {
      std::vector<Task> tasks;
      Planner P(*l, tasks);
      if (trans) P.bsolve_h2(0, B_X);
      else P.fsolve_h2(0, B_X);
      upload_tasks(*l, tl, tasks, P.aux);
    }
    prec_gather(l, r, nrhs);
    run_tasks(*l, tl, prec_threads(*l, nrhs));
    prec_scatter(l, z, nrhs);
    check_device_error(*l);
  });
}

h2_status h2_precond_config(h2_mat l, int32_t nrhs, int32_t threads) {
  return guarded([&] {
    require_ok(l);
    REQUIRE(l->lower && !l->inverse, "h2_precond_config needs a Cholesky factor");
    REQUIRE(nrhs >= 1 && nrhs <= H2_MAX_COLS, "nrhs out of range");
    REQUIRE(threads == 0 || std::find(std::begin(PREC_SHAPES), std::end(PREC_SHAPES), threads) !=
                                std::end(PREC_SHAPES),
            "threads must be 0, 128, 256 or 512");
    l->prec_nt[nrhs] = threads;
  });
}

// Key of a tuning result: the device's architecture and the shape of the
// substitution work (unknowns, clusters, blocks, stored values, columns).
static std::string tune_key(h2_mat_s &l, int nrhs) {
  hipDeviceProp_t pr;
  HIPCHK(hipGetDeviceProperties(&pr, l.ctx->device));
  const h2_ctree_s &ct = *l.bt->ct;
  char buf[256];
  std::snprintf(buf, sizeof buf, "precond/%s/n%ld/c%ld/a%d/b%d/v%lld/r%d", pr.gcnArchName, (long)ct.n,
                (long)ct.nc, l.nadm, l.nnear, (long long)mat_stored_values(l, nullptr, nullptr), nrhs);
  for (char *c = buf; *c; ++c)
    if (*c == ' ' || *c == ':') *c = '_';
  return buf;
}

h2_status h2_autotune_precond(h2_mat l, int32_t nrhs, int32_t reps, const char *cache_path, int32_t *threads,
                              double *ms_per_apply, int32_t *from_cache, double *ms_by_shape) {
  return guarded([&] {
    require_ok(l);
    REQUIRE(l->lower && !l->inverse, "h2_autotune_precond needs a Cholesky factor");
    REQUIRE(nrhs >= 1 && nrhs <= H2_MAX_COLS, "nrhs out of range");
    REQUIRE(reps >= 1 && reps <= 1000, "reps must be in [1, 1000]");
    const std::string key = tune_key(*l, nrhs);
    if (from_cache) *from_cache = 0;
    if (ms_by_shape)
      for (int i = 0; i < 3; ++i) ms_by_shape[i] = 0.0;
    if (cache_path && *cache_path) {
      if (FILE *f = std::fopen(cache_path, "r")) {
        char k[256];
        int t = 0;
        double ms = 0.0;
        int best = 0;
        double best_ms = 0.0;
        while (std::fscanf(f, "%255s %d %lf", k, &t, &ms) == 3)
          if (key == k && std::find(std::begin(PREC_SHAPES), std::end(PREC_SHAPES), t) != std::end(PREC_SHAPES)) {
            best = t;       // the last entry of a key wins
            best_ms = ms;
          }
        std::fclose(f);
        if (best > 0) {
          l->prec_nt[nrhs] = best;
          if (threads) *threads = best;
          if (ms_per_apply) *ms_per_apply = best_ms;
          if (from_cache) *from_cache = 1;
          return;
        }
      }
    }
    const h2_ctree_s &ct = *l->bt->ct;
    hipStream_t s = l->ctx->stream;
    const size_t len = (size_t)ct.n * nrhs;
    Dev<double> r, z;
    r.alloc_on(len, s);
    z.alloc_on(len, s);
    hipLaunchKernelGGL(k_fill_double, dim3(grid_for((long)len)), dim3(256), 0, s, r.p, (int)len, 1.0);
    HIPCHK(hipGetLastError());
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    struct Events {
      hipEvent_t a, b;
      ~Events() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } ev{e0, e1};
    const int saved = l->prec_nt[nrhs];
    int best = 0;
    double best_ms = 0.0;
    try {
      for (int si = 0; si < 3; ++si) {
        const int t = PREC_SHAPES[si];
        l->prec_nt[nrhs] = t;
        precond_device(l, r.p, z.p, nrhs);      // warm-up (and plans the list once)
        HIPCHK(hipEventRecord(e0, s));
        for (int i = 0; i < reps; ++i) precond_device(l, r.p, z.p, nrhs);
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        const double per = (double)ms / reps;
        if (ms_by_shape) ms_by_shape[si] = per;
        if (best == 0 || per < best_ms) { best = t; best_ms = per; }
      }
    } catch (...) {
      l->prec_nt[nrhs] = saved;
      throw;
    }
    check_device_error(*l);
    l->prec_nt[nrhs] = best;
    if (threads) *threads = best;
    if (ms_per_apply) *ms_per_apply = best_ms;
    if (cache_path && *cache_path) {
      FILE *f = std::fopen(cache_path, "a");
      REQUIRE(f != nullptr, "cannot append to the tuning cache file");
      std::fprintf(f, "%s %d %.6f\n", key.c_str(), best, best_ms);
      std::fclose(f);
    }
  });
}

h2_status h2_lr_solve(h2_mat f, const double *r, double *z, int32_t nrhs) {
  return guarded([&] {
    require_ok(f);
    REQUIRE(f->lr, "h2_lr_solve needs a matrix factorised by h2_lr");
    REQUIRE(r && z, "null vector");
    REQUIRE(nrhs >= 1 && nrhs <= H2_MAX_COLS, "nrhs out of range");
    if (!f->lrsolve.built) {
      std::vector<Task> tasks;
      Planner P(*f, tasks);
      P.fsolve_unit(0, B_X);
      P.bsolve_upper(0, B_X);
      upload_tasks(*f, f->lrsolve, tasks, P.aux);
    }
    prec_gather(f, r, nrhs);
    run_tasks(*f, f->lrsolve);
    prec_scatter(f, z, nrhs);
    check_device_error(*f);
  });
}

h2_status h2_csr_create(h2_ctx ctx, int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                        h2_csr *out) {
  return guarded([&] {
    REQUIRE(ctx && rowptr && col && val && out, "null argument");
    REQUIRE(n >= 1, "n must be positive");
    REQUIRE(ctx->device >= 0, "a host-only context cannot hold device data");
    auto a = std::make_unique<h2_csr_s>();
    a->ctx = ctx; a->n = n;
    const int64_t nnz = rowptr[n];
    std::vector<int64_t> rp(rowptr, rowptr + n + 1);
    std::vector<int> ci(col, col + nnz);
    std::vector<double> v(val, val + nnz);
    a->rp.upload(rp, ctx->stream); a->ci.upload(ci, ctx->stream); a->v.upload(v, ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *out = a.release();
  });
}

h2_status h2_csr_destroy(h2_csr a) {
  delete a;
  return H2_OK;
}

h2_status h2_spmv(h2_csr a, const double *x, double *y) {
  return guarded([&] {
    REQUIRE(a && x && y, "null argument");
    hipLaunchKernelGGL(k_spmv, dim3(grid_for(a->n)), dim3(256), 0, a->ctx->stream, (int)a->n, a->rp.p, a->ci.p,
                       a->v.p, x, y);
    HIPCHK(hipGetLastError());
  });
}

}  // extern "C"

static void pcg_batched(h2_csr *as, h2_mat *ls, const double *const *bs, double *const *xs, const int32_t *nrhs,
                        int32_t count, double rtol, int32_t maxit, int32_t *iters, double *relres,
                        h2_status *status, bool graph) {
  REQUIRE(as && bs && xs, "null argument");
  REQUIRE(maxit >= 1 && rtol >= 0.0, "bad maxit or rtol");
  std::vector<h2_mat_s *> ms = batch_members(ls, count, graph ? "h2_pcg_batched_graph" : "h2_pcg_batched");
  hipStream_t s = ms[0]->ctx->stream;
  const int NP = 256;   // partial sums of the dot products
  // one CG iteration state per column; a system's columns share its
  // preconditioner launches
  struct Col {
    const double *b; double *x, *r, *z, *p, *q, *part, *sc;
    double nb, rel; int it; bool active, conv;
  };
  struct Sys {
    h2_csr_s *a; h2_mat_s *l; int n, g, k, c0; double *R, *Z;
  };
  std::vector<Sys> sys(count);
  std::vector<Col> col;
  for (int i = 0; i < count; ++i) {
    Sys &y = sys[i];
    y.a = as[i]; y.l = ms[i];
    REQUIRE(y.a && bs[i] && xs[i], "null argument");
    REQUIRE(y.a->n == y.l->bt->ct->n, "size mismatch");
    y.n = (int)y.a->n;
    y.k = nrhs ? nrhs[i] : 1;
    REQUIRE(y.k >= 1 && y.k <= BC, "nrhs must be in [1, H2_MAX_COLS]");
    y.g = grid_for(y.n);
    const size_t need = (size_t)(4 * y.n + NP + 8) * y.k;
    if (y.l->d_pcg.n < need) y.l->d_pcg.alloc_on(need, y.l->stream);
    double *base = y.l->d_pcg.p;
    y.R = base;
    y.Z = y.R + (size_t)y.n * y.k;
    double *P = y.Z + (size_t)y.n * y.k, *Q = P + (size_t)y.n * y.k, *PART = Q + (size_t)y.n * y.k;
    double *SC = PART + (size_t)NP * y.k;
    y.c0 = (int)col.size();
    for (int c = 0; c < y.k; ++c) {
      const size_t o = (size_t)c * y.n;
      col.push_back(Col{bs[i] + o, xs[i] + o, y.R + o, y.Z + o, P + o, Q + o, PART + (size_t)c * NP,
                        SC + 8 * c, 0.0, 0.0, 0, true, false});
    }
    prec_list(y.l);
    sync_env(*y.l);
  }
  const int ncol = (int)col.size();
  if (status)
    for (int c = 0; c < ncol; ++c) status[c] = H2_OK;
  auto sys_active = [&](const Sys &y) {
    for (int c = 0; c < y.k; ++c)
      if (col[y.c0 + c].active) return true;
    return false;
  };
  auto dot = [&](const Sys &y, Col &c, const double *u, const double *v, double *dst) {
    hipLaunchKernelGGL(k_dot_partial, dim3(NP), dim3(256), 0, s, y.n, u, v, c.part);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, s, NP, c.part, dst);
  };
  std::vector<double> hs(ncol);
  auto read_scalars = [&](int slot) {     // sc[slot] of every active column
    for (int c = 0; c < ncol; ++c)
      if (col[c].active) HIPCHK(hipMemcpyAsync(&hs[c], col[c].sc + slot, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  };
  std::vector<BatchItem> items(count);
  struct ItemsGuard {
    Dev<BatchItem> *d; hipStream_t s;
    ~ItemsGuard() { (void)hipStreamSynchronize(s); items_release(d); }
  } guard{items_acquire(count), s};
  Dev<BatchItem> &d_items = *guard.d;
  // Z = (L L^*)^{-1} R for every system with an active column: one launch,
  // one workgroup per system, all its columns at once
  auto precond_all = [&]() {
    for (int i = 0; i < count; ++i) {
      Sys &y = sys[i];
      const bool act = sys_active(y);
      const TaskList &tl = y.l->prec;
      items[i] = BatchItem{tl.d.p, y.l->d_env.p, tl.aux.p, act ? tl.count : 0, 0};
      if (act) prec_gather(y.l, y.R, y.k);
    }
    int nt = 0;   // one launch shape for all: the largest tuned one
    for (const Sys &y : sys) nt = std::max(nt, prec_threads(*y.l, y.k));
    launch_batch(d_items, items, nt, s);
    for (Sys &y : sys)
      if (sys_active(y)) prec_scatter(y.l, y.Z, y.k);
  };
  for (Sys &y : sys)
    for (int c = 0; c < y.k; ++c) {
      Col &t = col[y.c0 + c];
      HIPCHK(hipMemsetAsync(t.x, 0, y.n * sizeof(double), s));
      HIPCHK(hipMemcpyAsync(t.r, t.b, y.n * sizeof(double), hipMemcpyDeviceToDevice, s));
      dot(y, t, t.b, t.b, t.sc + 4);
    }
  read_scalars(4);
  for (int c = 0; c < ncol; ++c) {
    col[c].nb = std::sqrt(hs[c]);
    if (col[c].nb == 0.0) { col[c].active = false; col[c].conv = true; }
  }
  precond_all();
  for (Sys &y : sys)
    for (int c = 0; c < y.k; ++c) {
      Col &t = col[y.c0 + c];
      if (!t.active) continue;
      HIPCHK(hipMemcpyAsync(t.p, t.z, y.n * sizeof(double), hipMemcpyDeviceToDevice, s));
      dot(y, t, t.r, t.z, t.sc + 0);
    }
  if (graph) {
    // One CG iteration of every column as a HIP graph, replayed until no
    // column is active: all columns per launch (k_bpcg_*), gated by flags
    // that the convergence test sets on the device, the preconditioner
    // launch gated per system.  Only kernels are captured.
    REQUIRE(ncol <= 65535, "too many right-hand sides for the graph form");
    std::vector<PcgCol> hc(ncol);
    std::vector<int> hctl(4 * (size_t)ncol + count + 1, 0);
    int *h_act = hctl.data(), *h_conv = h_act + 2 * ncol, *h_sys = h_act + 3 * ncol;
    int gx = 1;
    for (int i = 0; i < count; ++i) {
      const Sys &y = sys[i];
      gx = std::max(gx, y.g);
      for (int c = 0; c < y.k; ++c) {
        const Col &t = col[y.c0 + c];
        hc[y.c0 + c] = PcgCol{y.a->rp.p, y.a->ci.p, y.a->v.p, t.x, t.r, t.z, t.p, t.q, t.part, t.sc, t.nb, y.n, i};
        h_act[y.c0 + c] = t.active ? 1 : 0;
        h_conv[y.c0 + c] = t.conv ? 1 : 0;
        if (t.active) h_sys[i] = 1;
      }
    }
    Dev<PcgCol> d_cols;
    Dev<int> d_ctl;
    Dev<double> d_rel;
    d_cols.alloc_on(ncol, s);
    d_ctl.alloc_on(hctl.size(), s);
    d_rel.alloc_on(ncol, s);
    HIPCHK(hipMemcpyAsync(d_cols.p, hc.data(), ncol * sizeof(PcgCol), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d_ctl.p, hctl.data(), hctl.size() * sizeof(int), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_fill_double, dim3(grid_for(ncol)), dim3(256), 0, s, d_rel.p, ncol, 0.0);
    const PcgCtl ctl{d_ctl.p, d_ctl.p + ncol, d_ctl.p + 2 * ncol, d_ctl.p + 3 * ncol, d_ctl.p + 3 * ncol + count,
                     d_rel.p};
    int nt = 0;
    for (int i = 0; i < count; ++i) {
      const Sys &y = sys[i];
      const TaskList &tl = y.l->prec;
      items[i] = BatchItem{tl.d.p, y.l->d_env.p, tl.aux.p, tl.count, 0, ctl.sys_act + i};
      nt = std::max(nt, prec_threads(*y.l, y.k));
    }
    HIPCHK(hipMemcpyAsync(d_items.p, items.data(), count * sizeof(BatchItem), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    struct GraphGuard {
      hipStream_t cs = nullptr; hipGraph_t g = nullptr; hipGraphExec_t x = nullptr; bool capturing = false;
      ~GraphGuard() {
        if (capturing) { hipGraph_t t = nullptr; (void)hipStreamEndCapture(cs, &t); if (t) (void)hipGraphDestroy(t); }
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
        if (cs) (void)hipStreamDestroy(cs);
      }
    } gg;
    // captured on a private stream (a legacy default stream cannot capture)
    HIPCHK(hipStreamCreateWithFlags(&gg.cs, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(gg.cs, hipStreamCaptureModeThreadLocal));
    gg.capturing = true;
    const hipStream_t c = gg.cs;
    const dim3 gv((unsigned)gx, (unsigned)ncol), gd((unsigned)NP, (unsigned)ncol);
    hipLaunchKernelGGL(k_bpcg_spmv, gv, dim3(256), 0, c, (const PcgCol *)d_cols.p, (const int *)ctl.act);
    hipLaunchKernelGGL(k_bpcg_dot_partial, gd, dim3(256), 0, c, (const PcgCol *)d_cols.p, (const int *)ctl.act,
                       (int)PCG_DOT_PQ);
    hipLaunchKernelGGL(k_bpcg_dot_final, dim3(ncol), dim3(256), 0, c, (const PcgCol *)d_cols.p,
                       (const int *)ctl.act, NP, 1);
    hipLaunchKernelGGL(k_bpcg_update_xr, gv, dim3(256), 0, c, (const PcgCol *)d_cols.p, (const int *)ctl.act);
    hipLaunchKernelGGL(k_bpcg_dot_partial, gd, dim3(256), 0, c, (const PcgCol *)d_cols.p, (const int *)ctl.act,
                       (int)PCG_DOT_RR);
    hipLaunchKernelGGL(k_bpcg_dot_final, dim3(ncol), dim3(256), 0, c, (const PcgCol *)d_cols.p,
                       (const int *)ctl.act, NP, 3);
    hipLaunchKernelGGL(k_bpcg_check, dim3(1), dim3(256), 0, c, (const PcgCol *)d_cols.p, ctl, ncol, count, rtol,
                       (int)maxit);
    for (const Sys &y : sys) {
      const h2_ctree_s &ct = *y.l->bt->ct;
      const long work = (long)ct.n * y.k;
      hipLaunchKernelGGL(k_gather, dim3(grid_for(work)), dim3(256), 0, c, (int)ct.n, 0, y.k, ct.d_perm.p,
                         (const double *)y.R, (long)ct.n, y.l->env.buf[B_X], y.l->d_bcols.p, (int)B_X);
    }
    hipLaunchKernelGGL(k_interp_batch, dim3((unsigned)count), dim3((unsigned)nt),
                       LDS_TOTAL_DOUBLES * sizeof(double), c, (const BatchItem *)d_items.p);
    for (const Sys &y : sys) {
      const h2_ctree_s &ct = *y.l->bt->ct;
      const long work = (long)ct.n * y.k;
      hipLaunchKernelGGL(k_scatter, dim3(grid_for(work)), dim3(256), 0, c, (int)ct.n, y.k, ct.d_perm.p,
                         (const double *)y.l->env.buf[B_X], y.Z, (long)ct.n, 1.0, 0.0);
    }
    hipLaunchKernelGGL(k_bpcg_dot_partial, gd, dim3(256), 0, c, (const PcgCol *)d_cols.p, (const int *)ctl.act,
                       (int)PCG_DOT_RZ);
    hipLaunchKernelGGL(k_bpcg_dot_final, dim3(ncol), dim3(256), 0, c, (const PcgCol *)d_cols.p,
                       (const int *)ctl.act, NP, 2);
    hipLaunchKernelGGL(k_bpcg_update_p, gv, dim3(256), 0, c, (const PcgCol *)d_cols.p, (const int *)ctl.act);
    hipLaunchKernelGGL(k_bpcg_next, dim3(grid_for(ncol)), dim3(256), 0, c, (const PcgCol *)d_cols.p,
                       (const int *)ctl.act, ncol);
    gg.capturing = false;
    HIPCHK(hipStreamEndCapture(c, &gg.g));
    HIPCHK(hipGetLastError());
    HIPCHK(hipGraphInstantiate(&gg.x, gg.g, nullptr, nullptr, 0));
    // every replay counts an iteration for each active column, so at most
    // maxit replays leave none active
    int nact = 1;
    for (int rep = 0; rep < maxit && nact > 0; ++rep) {
      HIPCHK(hipGraphLaunch(gg.x, s));
      HIPCHK(hipMemcpyAsync(&nact, ctl.nact, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    std::vector<int> h_it(ncol), h_cv(ncol);
    std::vector<double> h_rel(ncol);
    HIPCHK(hipMemcpyAsync(h_it.data(), ctl.it, ncol * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(h_cv.data(), ctl.conv, ncol * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(h_rel.data(), ctl.rel, ncol * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int k = 0; k < ncol; ++k) {
      col[k].it = h_it[k];
      col[k].conv = h_cv[k] != 0;
      col[k].rel = h_rel[k];
      col[k].active = false;
    }
  } else for (;;) {
    bool any = false;
    for (Sys &y : sys)
      for (int c = 0; c < y.k; ++c) {
        Col &t = col[y.c0 + c];
        if (!t.active) continue;
        any = true;
        hipLaunchKernelGGL(k_spmv, dim3(y.g), dim3(256), 0, s, y.n, y.a->rp.p, y.a->ci.p, y.a->v.p, t.p, t.q);
        ++t.it;
        dot(y, t, t.p, t.q, t.sc + 1);
        hipLaunchKernelGGL(k_pcg_update_xr, dim3(y.g), dim3(256), 0, s, y.n, t.sc, t.p, t.q, t.x, t.r);
        dot(y, t, t.r, t.r, t.sc + 3);
      }
    if (!any) break;
    read_scalars(3);
    any = false;
    for (Col &t : col) {
      if (!t.active) continue;
      t.rel = std::sqrt(hs[&t - col.data()]) / t.nb;
      if (t.rel <= rtol) { t.conv = true; t.active = false; }
      else if (t.it >= maxit) t.active = false;
      any = any || t.active;
    }
    if (!any) break;
    precond_all();
    for (Sys &y : sys)
      for (int c = 0; c < y.k; ++c) {
        Col &t = col[y.c0 + c];
        if (!t.active) continue;
        dot(y, t, t.r, t.z, t.sc + 2);
        hipLaunchKernelGGL(k_pcg_update_p, dim3(y.g), dim3(256), 0, s, y.n, t.sc, t.z, t.p);
        hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, s, t.sc + 0, t.sc + 2);
      }
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  for (int c = 0; c < ncol; ++c) {
    if (iters) iters[c] = col[c].it;
    if (relres) relres[c] = col[c].rel;
  }
  std::vector<h2_status> sst(count, H2_OK);
  try {
    batch_errors(ms, sst.data());
  } catch (const H2Error &) {
    if (status)
      for (int i = 0; i < count; ++i)
        for (int c = 0; c < sys[i].k; ++c) status[sys[i].c0 + c] = sst[i];
    throw;
  }
  int bad = -1;
  for (int c = 0; c < ncol; ++c)
    if (!col[c].conv) {
      if (status) status[c] = H2_ERR_NOT_CONVERGED;
      if (bad < 0) bad = c;
    }
  if (bad >= 0)
    throw H2Error(H2_ERR_NOT_CONVERGED,
                  "PCG did not reach the tolerance (first: right-hand side " + std::to_string(bad) + ")");
}

extern "C" {

h2_status h2_pcg_batched(h2_csr *as, h2_mat *ls, const double *const *bs, double *const *xs,
                         const int32_t *nrhs, int32_t count, double rtol, int32_t maxit, int32_t *iters,
                         double *relres, h2_status *status) {
  return guarded([&] { pcg_batched(as, ls, bs, xs, nrhs, count, rtol, maxit, iters, relres, status, false); });
}

h2_status h2_pcg_batched_graph(h2_csr *as, h2_mat *ls, const double *const *bs, double *const *xs,
                               const int32_t *nrhs, int32_t count, double rtol, int32_t maxit, int32_t *iters,
                               double *relres, h2_status *status) {
  return guarded([&] { pcg_batched(as, ls, bs, xs, nrhs, count, rtol, maxit, iters, relres, status, true); });
}

}  // extern "C"

extern "C" {

// PCG body shared by h2_pcg and h2_pcg_noalloc.  work: 4n + PCG_PART + 8
// doubles (r, z, p, q, dot partial sums, scalars).  fill_kernel: clear x
// with a fill kernel instead of hipMemsetAsync.
constexpr int PCG_PART = 256;
static void pcg_run(h2_csr a, h2_mat l, const double *b, double *x, double rtol, int32_t maxit, int32_t *iters,
                    double *relres, double *work, bool fill_kernel) {
  const int n = (int)a->n;
  hipStream_t s = l->ctx->stream;
  const int NP = PCG_PART;
  double *r = work, *z = r + n, *p = z + n, *q = p + n, *part = q + n, *sc = part + NP;
  const int g = grid_for(n);
  auto dot = [&](const double *u, const double *v, double *dst) {
    hipLaunchKernelGGL(k_dot_partial, dim3(NP), dim3(256), 0, s, n, u, v, part);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, s, NP, part, dst);
  };
  auto host_scalar = [&](const double *dsrc) {
    double v = 0.0;
    HIPCHK(hipMemcpyAsync(&v, dsrc, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return v;
  };
  if (fill_kernel) hipLaunchKernelGGL(k_fill_double, dim3(g), dim3(256), 0, s, x, n, 0.0);
  else HIPCHK(hipMemsetAsync(x, 0, n * sizeof(double), s));
  HIPCHK(hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  dot(b, b, sc + 4);
  const double nb = std::sqrt(host_scalar(sc + 4));
  int it = 0;
  double rel = 0.0;
  if (nb == 0.0) {
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    return;
  }
  precond_device(l, r, z, 1);
  HIPCHK(hipMemcpyAsync(p, z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  dot(r, z, sc + 0);
  bool conv = false;
  while (it < maxit) {
    hipLaunchKernelGGL(k_spmv, dim3(g), dim3(256), 0, s, n, a->rp.p, a->ci.p, a->v.p, p, q);
    ++it;
    dot(p, q, sc + 1);
    hipLaunchKernelGGL(k_pcg_update_xr, dim3(g), dim3(256), 0, s, n, sc, p, q, x, r);
    dot(r, r, sc + 3);
    rel = std::sqrt(host_scalar(sc + 3)) / nb;
    if (rel <= rtol) { conv = true; break; }
    precond_device(l, r, z, 1);
    dot(r, z, sc + 2);
    hipLaunchKernelGGL(k_pcg_update_p, dim3(g), dim3(256), 0, s, n, sc, z, p);
    hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, s, sc + 0, sc + 2);
  }
  HIPCHK(hipGetLastError());
  check_device_error(*l);
  if (iters) *iters = it;
  if (relres) *relres = rel;
  if (!conv) throw H2Error(H2_ERR_NOT_CONVERGED, "PCG did not reach the tolerance");
}

static void pcg_check_args(h2_csr a, h2_mat l, const double *b, double *x, double rtol, int32_t maxit) {
  REQUIRE(a && b && x, "null argument");
  require_ok(l);
  REQUIRE(l->lower, "h2_pcg needs a Cholesky factor");
  REQUIRE(a->n == l->bt->ct->n, "size mismatch");
  REQUIRE(maxit >= 1 && rtol >= 0.0, "bad maxit or rtol");
}

h2_status h2_pcg(h2_csr a, h2_mat l, const double *b, double *x, double rtol, int32_t maxit, int32_t *iters,
                 double *relres) {
  return guarded([&] {
    pcg_check_args(a, l, b, x, rtol, maxit);
    const size_t need = (size_t)4 * a->n + PCG_PART + 8;
    if (l->d_pcg.n < need) l->d_pcg.alloc_on(need, l->stream);
    pcg_run(a, l, b, x, rtol, maxit, iters, relres, l->d_pcg.p, false);
  });
}

h2_status h2_pcg_noalloc(h2_csr a, h2_mat l, const double *b, double *x, double rtol, int32_t maxit,
                         int32_t *iters, double *relres) {
  return guarded([&] {
    pcg_check_args(a, l, b, x, rtol, maxit);
    REQUIRE(a->n <= H2_NOALLOC_MAX_N, "h2_pcg_noalloc: n = " + std::to_string(a->n) +
                                          " exceeds the fixed work area of H2_NOALLOC_MAX_N = " +
                                          std::to_string((long)H2_NOALLOC_MAX_N) + " unknowns");
    const bool planned = l->inverse ? l->prec_inv.built : l->prec.built;
    REQUIRE(planned && l->d_env.p,
            "h2_pcg_noalloc: the preconditioner of this factor is not planned yet (its task list is "
            "allocated by the first h2_precond or h2_pcg call on the factor)");
    pcg_run(a, l, b, x, rtol, maxit, iters, relres, noalloc_scratch(l->ctx->device), true);
  });
}

}  // extern "C"
