// C ABI of the HODLR library: argument checking, the integer plan (tree,
// row tiles, reduction segments), device memory, and the level-synchronous
// orchestration of the kernels (Section III-C: the cluster tree is the task
// graph, nodes of one level are independent, each level waits for the one
// below).  Every launch goes to the caller's stream; the only host
// synchronisations are the singularity verdict of a factorization and the
// residual norm of each refinement step.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <climits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"

using namespace hodlr;

// ---------------------------------------------------------------------------
// per-kernel timing with HIP events on the launch stream
// ---------------------------------------------------------------------------
namespace {
struct TimeRec {
  const char* name;
  hipEvent_t e0, e1;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<TimeRec> g_recs;
std::vector<hipEvent_t> g_pool;
std::map<std::string, std::pair<double, int64_t>> g_tot;

hipEvent_t pool_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  hipEventCreate(&e);
  return e;
}
void drain_records() {
  for (auto& r : g_recs) {
    float ms = 0.f;
    hipEventSynchronize(r.e1);
    hipEventElapsedTime(&ms, r.e0, r.e1);
    auto& t = g_tot[r.name];
    t.first += ms;
    t.second += 1;
    g_pool.push_back(r.e0);
    g_pool.push_back(r.e1);
  }
  g_recs.clear();
}

struct TimerScope {
  hipStream_t s;
  const char* name;
  hipEvent_t e1 = nullptr;
  hipEvent_t e0 = nullptr;
  bool on;
  TimerScope(hipStream_t s_, const char* n) : s(s_), name(n) {
    std::lock_guard<std::mutex> g(g_tmu);
    on = g_timing;
    if (on) {
      e0 = pool_event();
      e1 = pool_event();
      hipEventRecord(e0, s);
    }
  }
  ~TimerScope() {
    if (!on) return;
    std::lock_guard<std::mutex> g(g_tmu);
    hipEventRecord(e1, s);
    g_recs.push_back({name, e0, e1});
    if (g_recs.size() > 4096) drain_records();
  }
};
}  // namespace

#define HL(name, call)                                     \
  do {                                                     \
    TimerScope _ts(st, name);                              \
    hipError_t _e = (call);                                \
    if (_e != hipSuccess) return hip_fail(_e, name);       \
  } while (0)

static hodlr_status hip_fail(hipError_t e, const char* what) {
  if (getenv("HODLR_VERBOSE")) fprintf(stderr, "hodlr: %s failed: %s\n", what, hipGetErrorString(e));
  return HODLR_ERR_HIP;
}

// ---------------------------------------------------------------------------
// plan and factor object
// ---------------------------------------------------------------------------
namespace {

struct DevMem {
  std::vector<void*> ptrs;
  size_t bytes = 0;
  template <typename X>
  hodlr_status alloc(X** p, size_t count) {
    *p = nullptr;
    if (count == 0) return HODLR_OK;
    void* q = nullptr;
    if (hipMalloc(&q, count * sizeof(X)) != hipSuccess) return HODLR_ERR_ALLOC;
    ptrs.push_back(q);
    bytes += count * sizeof(X);
    *p = static_cast<X*>(q);
    return HODLR_OK;
  }
  void release() {
    for (void* p : ptrs) hipFree(p);
    ptrs.clear();
    bytes = 0;
  }
};

// Reduction plan of a product whose node level is p, computed on tiles of level q >= p.
// Tile partials are summed in stages of at most kSegTiles items (fixed order) until every
// node has a single sum left, which the coupling kernels read.
struct ProdStage {
  int nsegs = 0;
  int maxy = 0;            // largest item count of a segment
  int2* d_desc = nullptr;  // per output segment: first input item, count
};
struct ProdPlan {
  int nnodes = 0;
  int maxcount = 0;
  std::vector<ProdStage> stages;  // empty: the coupling kernels read tile partials directly
  size_t buf_items[2] = {0, 0};   // ping-pong regions of the segment buffer, in items
  int32_t* d_seg_start = nullptr;
};

// Solve-side workspace of one stream: tile partials, segment sums, W, the
// compute-type copy of the right-hand sides, refinement vectors, projection
// trees and norms for up to `nrhs` columns.  Calls on different streams use
// different workspaces, so they may run concurrently on one factorization;
// calls on one stream are ordered by the stream.
struct Workspace {
  hipStream_t stream = nullptr;
  std::mutex mu;  // one host call at a time on this stream
  DevMem mem;
  int nrhs = -1;
  void* sP = nullptr;
  void* sseg = nullptr;
  void* sw = nullptr;
  void* sx = nullptr;      // compute-type copy of the right-hand sides
  double* rx = nullptr;    // refinement: iterate x
  double* rr = nullptr;    // refinement: residual
  double* tree = nullptr;  // matvec projection tree
  double* tree2 = nullptr;
  double* nrm = nullptr;       // norms: part | b2 | r2 | rinf
  double* ld = nullptr;        // log-determinant: per-item logs | per-item parities | result
  hipEvent_t done = nullptr;   // recorded after the last call's work on `stream`
};

}  // namespace

struct hodlr_factors {
  // shape
  int64_t n = 0;
  int L = 0;
  int nleaf = 1;
  int m_max = 0;
  int ldl = 0;  // leaf factor block size: m_max rounded up to a multiple of 16
  int R = 0;
  std::vector<int64_t> off;
  std::vector<int> ranks;  // r_1..r_L
  std::vector<int> Rp;     // R_0..R_L
  hodlr_dtype storage = HODLR_F64, compute = HODLR_F64;
  int inplace = 0;  // HODLR_INPLACE: LU in the caller's D, Y in the caller's U
  // the caller's matrix
  const void *D = nullptr, *U = nullptr, *V = nullptr;
  int64_t ldd = 0, ldu = 0, ldv = 0;
  // device plan
  DevMem mem;
  int64_t* d_off = nullptr;
  int32_t* d_rpre = nullptr;
  std::vector<Tile*> d_tiles;                 // per tile level q = 0..L
  std::vector<int> ntiles;                    // per q
  std::vector<std::vector<Tile>> h_tiles;     // per q (host copy)
  std::vector<int> tiles_aligned;             // per q: bit 0 every tile height % 16 == 0, bit 1 % 32 == 0
  int64_t ldy = 0, gsy = 256;                 // Y layout: row i, column c at (i >> 8) * gsy + (i & 255) + c * ldy
  std::vector<std::vector<int>> tile_start;   // per q, 2^q + 1
  std::map<std::pair<int, int>, ProdPlan> prods;
  // factors (T = compute element type)
  size_t tsize = 8;
  void* lu = nullptr;
  int64_t lul = 0;  // leading dimension of the leaf factors (ldl, or ldd in place)
  int32_t* piv = nullptr;
  int32_t* perm = nullptr;
  void* udinv = nullptr;
  void* invl = nullptr;  // leaf LU scratch: inverted diagonal blocks of L
  void* Y = nullptr;
  std::vector<int64_t> koff, kvoff, kioff;  // per parent level p: offsets of K blocks / K vectors / K inverses
  void* Klu = nullptr;
  int32_t* Kpiv = nullptr;
  int32_t* Kperm = nullptr;
  void* Kud = nullptr;
  void* Kinv = nullptr;  // inverted 16 x 16 diagonal blocks of the K factors
  // factor workspace
  void* W = nullptr;
  void* P = nullptr;
  void* segbuf = nullptr;
  unsigned long long* d_info = nullptr;
  // solve / matvec / refinement workspaces, one per stream, grown on demand
  std::mutex mu;  // guards wsmap; held by refactor for its whole enqueue
  std::map<hipStream_t, std::unique_ptr<Workspace>> wsmap;
  hipEvent_t ready = nullptr;  // recorded after the factorization's last kernel
  bool singular = false;       // the last factorization met an exactly zero pivot
  // allocation-free solves (hodlr_solve_noalloc): the device the factors live
  // on, and the completion of the last such call (refactor and destroy wait on it)
  int device = 0;
  std::mutex na_mu;
  hipEvent_t na_done = nullptr;
  // complex matrices: the factors are those of the real embedding, whose
  // D, U, V the factorization owns here (n, off, ranks are the embedded ones)
  int cplx = 0;
  DevMem emb;
};

namespace {

int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

hodlr_status validate(const hodlr_matrix* A, std::vector<int64_t>& off, std::vector<int>& ranks, int& m_max) {
  if (!A || A->n < 1 || A->levels < 0 || A->levels > HODLR_MAX_LEVELS) return HODLR_ERR_ARG;
  const int L = A->levels;
  const int64_t nl = int64_t(1) << L;
  if (nl > A->n) return HODLR_ERR_ARG;
  off.assign(nl + 1, 0);
  if (A->leaf_offsets) {
    for (int64_t i = 0; i <= nl; ++i) off[i] = A->leaf_offsets[i];
    if (off[0] != 0 || off[nl] != A->n) return HODLR_ERR_ARG;
    for (int64_t i = 0; i < nl; ++i)
      if (off[i + 1] <= off[i]) return HODLR_ERR_ARG;
  } else {
    if (A->n % nl) return HODLR_ERR_ARG;
    for (int64_t i = 0; i <= nl; ++i) off[i] = i * (A->n / nl);
  }
  m_max = 0;
  for (int64_t i = 0; i < nl; ++i) m_max = (int)std::max<int64_t>(m_max, off[i + 1] - off[i]);
  if (m_max > HODLR_MAX_LEAF) return HODLR_ERR_UNSUPPORTED;
  ranks.assign(L, 0);
  if (L > 0 && !A->ranks) return HODLR_ERR_ARG;
  for (int l = 0; l < L; ++l) {
    if (A->ranks[l] < 0) return HODLR_ERR_ARG;
    if (A->ranks[l] > HODLR_MAX_RANK) return HODLR_ERR_UNSUPPORTED;
    ranks[l] = A->ranks[l];
  }
  // every level-l node must hold at least r_l rows (its generators are |I_a| x r_l
  // with r_l independent columns); node sizes by pairwise sums from the leaves
  {
    std::vector<int64_t> sz(nl);
    for (int64_t i = 0; i < nl; ++i) sz[i] = off[i + 1] - off[i];
    for (int l = L; l >= 1; --l) {
      int64_t mn = INT64_MAX;
      for (int64_t i = 0; i < (int64_t(1) << l); ++i) mn = std::min(mn, sz[i]);
      if (ranks[l - 1] > mn) return HODLR_ERR_ARG;
      for (int64_t i = 0; i < (int64_t(1) << (l - 1)); ++i) sz[i] = sz[2 * i] + sz[2 * i + 1];
    }
  }
  if (A->dtype != HODLR_F64 && A->dtype != HODLR_F32) return HODLR_ERR_ARG;
  int R = 0;
  for (int r : ranks) R += r;
  if (!A->D || A->ldd < A->n) return HODLR_ERR_ARG;
  if (R > 0 && (!A->U || !A->V || A->ldu < A->n || A->ldv < A->n)) return HODLR_ERR_ARG;
  return HODLR_OK;
}

// tiles of level q: every level-q node split into runs of <= kTileRows rows
void build_tiles(hodlr_factors* F, int q, std::vector<Tile>& out, std::vector<int>& start) {
  const int per = 1 << (F->L - q);
  const int nn = 1 << q;
  start.assign(nn + 1, 0);
  out.clear();
  for (int i = 0; i < nn; ++i) {
    start[i] = (int)out.size();
    const int64_t s = F->off[(int64_t)i * per], e = F->off[(int64_t)(i + 1) * per];
    for (int64_t r = s; r < e; r += kTileRows) out.push_back(Tile{r, (int32_t)std::min<int64_t>(kTileRows, e - r), i});
  }
  start[nn] = (int)out.size();
}

hodlr_status make_prod(hodlr_factors* F, int q, int p, hipStream_t st) {
  auto key = std::make_pair(q, p);
  if (F->prods.count(key)) return HODLR_OK;
  ProdPlan pp;
  pp.nnodes = 1 << p;
  const int stride = 1 << (q - p);
  const std::vector<int>& ts = F->tile_start[q];
  // items of each node: initially its tiles
  std::vector<int> start(pp.nnodes + 1);
  for (int i = 0; i <= pp.nnodes; ++i) start[i] = ts[i * stride];
  for (int i = 0; i < pp.nnodes; ++i) pp.maxcount = std::max(pp.maxcount, start[i + 1] - start[i]);
  int stage = 0;
  while (true) {
    int mx = 0;
    for (int i = 0; i < pp.nnodes; ++i) mx = std::max(mx, start[i + 1] - start[i]);
    if (mx <= 1) break;  // reduced to one item per node: the coupling kernels read plain sums
    std::vector<int2> desc;
    std::vector<int> nstart(pp.nnodes + 1);
    for (int i = 0; i < pp.nnodes; ++i) {
      nstart[i] = (int)desc.size();
      for (int t = start[i]; t < start[i + 1]; t += kSegTiles)
        desc.push_back(int2{t, std::min(kSegTiles, start[i + 1] - t)});
    }
    nstart[pp.nnodes] = (int)desc.size();
    ProdStage ps;
    ps.nsegs = (int)desc.size();
    for (const int2& d : desc) ps.maxy = std::max(ps.maxy, d.y);
    hodlr_status s = F->mem.alloc(&ps.d_desc, desc.size());
    if (s) return s;
    if (hipMemcpy(ps.d_desc, desc.data(), desc.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess)
      return HODLR_ERR_HIP;
    pp.buf_items[stage & 1] = std::max(pp.buf_items[stage & 1], desc.size());
    pp.stages.push_back(ps);
    start = nstart;
    ++stage;
  }
  hodlr_status s = F->mem.alloc(&pp.d_seg_start, start.size());
  if (s) return s;
  if (hipMemcpy(pp.d_seg_start, start.data(), start.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
    return HODLR_ERR_HIP;
  F->prods[key] = pp;
  (void)st;
  return HODLR_OK;
}

// tile level on which the product of node level p is computed
int fwd_prod_tiles(const hodlr_factors* F, int p) { return p == F->L ? F->L : p + 1; }
int adj_prod_tiles(const hodlr_factors*, int p) { return p; }

hodlr_status plan(hodlr_factors* F) {
  const int L = F->L;
  F->d_tiles.assign(L + 1, nullptr);
  F->ntiles.assign(L + 1, 0);
  F->tiles_aligned.assign(L + 1, 0);
  F->h_tiles.assign(L + 1, {});
  F->tile_start.assign(L + 1, {});
  std::vector<Tile> tl;
  for (int q = 0; q <= L; ++q) {
    build_tiles(F, q, tl, F->tile_start[q]);
    F->ntiles[q] = (int)tl.size();
    F->h_tiles[q] = tl;
    F->tiles_aligned[q] = 3;
    for (const Tile& t : tl)
      if (t.nrows % 16) F->tiles_aligned[q] = 0;
      else if (t.nrows % 32) F->tiles_aligned[q] &= 1;
    hodlr_status s = F->mem.alloc(&F->d_tiles[q], tl.size());
    if (s) return s;
    if (hipMemcpy(F->d_tiles[q], tl.data(), tl.size() * sizeof(Tile), hipMemcpyHostToDevice) != hipSuccess)
      return HODLR_ERR_HIP;
  }
  for (int p = 1; p <= L; ++p) {
    hodlr_status s = make_prod(F, fwd_prod_tiles(F, p), p, nullptr);
    if (s) return s;
    s = make_prod(F, adj_prod_tiles(F, p), p, nullptr);
    if (s) return s;
  }
  return HODLR_OK;
}

size_t tsz(hodlr_dtype c) { return c == HODLR_F64 ? 8 : 4; }

// leading dimension of a stored K factor: 2r rounded up to 16
int kpad(int r) { return (2 * r + 15) & ~15; }

hodlr_status allocate_factors(hodlr_factors* F) {
  DevMem& M = F->mem;
  const int L = F->L;
  const size_t ts = F->tsize;
  hodlr_status s;
  if ((s = M.alloc(&F->d_off, F->off.size()))) return s;
  if (hipMemcpy(F->d_off, F->off.data(), F->off.size() * 8, hipMemcpyHostToDevice) != hipSuccess) return HODLR_ERR_HIP;
  std::vector<int32_t> rp(F->Rp.begin(), F->Rp.end());
  if ((s = M.alloc(&F->d_rpre, rp.size()))) return s;
  if (hipMemcpy(F->d_rpre, rp.data(), rp.size() * 4, hipMemcpyHostToDevice) != hipSuccess) return HODLR_ERR_HIP;
  if ((s = plan(F))) return s;
  unsigned char* b;
  const size_t nl = F->nleaf, mm = F->ldl;
  if (F->inplace) {
    F->lu = const_cast<void*>(F->D);  // the leaf factors overwrite the caller's D
    F->lul = F->ldd;
  } else {
    if ((s = M.alloc(&b, nl * mm * mm * ts))) return s;
    F->lu = b;
    F->lul = F->ldl;
  }
  if ((s = M.alloc(&F->piv, nl * mm))) return s;
  if ((s = M.alloc(&F->perm, nl * mm))) return s;
  if ((s = M.alloc(&b, nl * mm * ts))) return s;
  F->udinv = b;
  if ((s = M.alloc(&b, nl * 2 * (mm / 16) * 256 * ts))) return s;
  F->invl = b;
  // Y in the row-group blocked layout (each 256-row group of all R columns
  // contiguous) when no leaf and no tile crosses a 256-row boundary, else
  // column-major with leading dimension N
  bool blocked = F->R > 0 && !F->inplace;  // in place, Y is column-major in the caller's U
  for (int a = 0; a < F->nleaf && blocked; ++a)
    if ((F->off[a] >> 8) != ((F->off[a + 1] - 1) >> 8)) blocked = false;
  for (int q = 0; q <= L && blocked; ++q)
    for (const Tile& t : F->h_tiles[q])
      if ((t.row0 >> 8) != ((t.row0 + t.nrows - 1) >> 8)) blocked = false;
  const int64_t ngroups = (F->n + 255) / 256;
  if (F->inplace) {
    F->Y = const_cast<void*>(F->U);
    F->ldy = F->ldu;
    F->gsy = 256;
  } else {
    F->ldy = blocked ? 256 : F->n;
    F->gsy = blocked ? 256 * (int64_t)F->R : 256;
    if ((s = M.alloc(&b, (size_t)(blocked ? ngroups * 256 : F->n) * F->R * ts))) return s;
    F->Y = b;
  }
  F->koff.assign(L + 1, 0);
  F->kvoff.assign(L + 1, 0);
  F->kioff.assign(L + 1, 0);
  int64_t kk = 0, kv = 0, ki = 0;
  size_t wmax = 0, pmax = 0, segmax = 0;
  for (int p = 0; p < L; ++p) {
    const int r = F->ranks[p];  // r_{p+1}
    const int kp = kpad(r);
    F->koff[p] = kk;
    F->kvoff[p] = kv;
    F->kioff[p] = ki;
    kk += (int64_t(1) << p) * kp * kp;
    kv += (int64_t(1) << p) * kp;
    ki += (int64_t(1) << p) * 2 * (kp / 16) * 256;
    wmax = std::max(wmax, (size_t)(int64_t(1) << p) * 2 * r * F->Rp[p]);
  }
  F->koff[L] = kk;
  F->kvoff[L] = kv;
  F->kioff[L] = ki;
  for (int p = 1; p <= L; ++p) {
    const int q = fwd_prod_tiles(F, p);
    const size_t elems = (size_t)F->ranks[p - 1] * F->Rp[p];
    pmax = std::max(pmax, (size_t)F->ntiles[q] * elems);
    const ProdPlan& pp = F->prods[{q, p}];
    segmax = std::max(segmax, (pp.buf_items[0] + pp.buf_items[1]) * elems);
  }
  if ((s = M.alloc(&b, (size_t)kk * ts))) return s;
  F->Klu = b;
  if ((s = M.alloc(&F->Kpiv, (size_t)kv))) return s;
  if ((s = M.alloc(&F->Kperm, (size_t)kv))) return s;
  if ((s = M.alloc(&b, (size_t)kv * ts))) return s;
  F->Kud = b;
  if ((s = M.alloc(&b, (size_t)ki * ts))) return s;
  F->Kinv = b;
  if ((s = M.alloc(&b, wmax * ts))) return s;
  F->W = b;
  if ((s = M.alloc(&b, pmax * ts))) return s;
  F->P = b;
  if ((s = M.alloc(&b, segmax * ts))) return s;
  F->segbuf = b;
  if ((s = M.alloc(&F->d_info, 2))) return s;
  if (hipEventCreateWithFlags(&F->ready, hipEventDisableTiming) != hipSuccess) return HODLR_ERR_HIP;
  if (hipEventCreateWithFlags(&F->na_done, hipEventDisableTiming) != hipSuccess) return HODLR_ERR_HIP;
  if (hipGetDevice(&F->device) != hipSuccess) return HODLR_ERR_HIP;
  return HODLR_OK;
}

template <typename T>
T* tp(void* p) {
  return static_cast<T*>(p);
}

// segments for the product of node level p on tile level q (reduces if needed)
template <typename T>
hodlr_status prod_segments(hodlr_factors* F, hipStream_t st, int q, int p, int64_t elems, T* P, T* segbuf,
                           const T** segs, const int32_t** seg_start) {
  const ProdPlan& pp = F->prods.at({q, p});
  const T* in = P;
  T* region[2] = {segbuf, segbuf + pp.buf_items[0] * elems};
  for (size_t k = 0; k < pp.stages.size(); ++k) {
    T* out = region[k & 1];
    HL("segment_reduce", launch_segment_reduce<T>(st, pp.stages[k].nsegs, pp.stages[k].d_desc, elems, in, out,
                                                  pp.stages[k].maxy));
    in = out;
  }
  *segs = in;
  *seg_start = pp.d_seg_start;
  return HODLR_OK;
}

// bf = 1: the leaf LU updates, the leaf solve and the level-pass products take
// bfloat16 operands (FP32 factors, accumulation, panels and K)
template <typename T, typename S>
hodlr_status run_factor(hodlr_factors* F, hipStream_t st, int bf) {
  const int L = F->L;
  const int64_t N = F->n;
  T* Y = tp<T>(F->Y);
  const S* D = static_cast<const S*>(F->D);
  const S* U = static_cast<const S*>(F->U);
  const S* V = static_cast<const S*>(F->V);
  if (hipMemsetAsync(F->d_info, 0xFF, 2 * sizeof(unsigned long long), st) != hipSuccess) return HODLR_ERR_HIP;
  HL("leaf_lu", (launch_leaf_lu<T, S>(st, F->nleaf, F->ldl, F->d_off, D, F->ldd, tp<T>(F->lu), F->lul, F->inplace,
                                      F->piv, F->perm, tp<T>(F->udinv), tp<T>(F->invl), F->d_info, bf)));
  if (F->R > 0)
    HL("leaf_trsm", (launch_leaf_trsm<T, S>(st, 0, F->nleaf, F->ldl, F->d_off, tp<T>(F->lu), F->lul, F->inplace,
                                            F->perm, tp<T>(F->invl), U, F->ldu, Y, F->ldy, F->R, 256, F->gsy, bf)));
  if (L > 0) {
    // products V^T Y for the children of level L-1 (the leaves)
    HL("level_pass", (launch_level_pass<T, T, S>(st, F->ntiles[L], F->d_tiles[L], F->tiles_aligned[L], Y, F->ldy, F->R,
                                                 (const T*)nullptr, F->ldy, 0, (const T*)nullptr, 0, 0, 0,
                                                 V + (int64_t)F->Rp[L - 1] * F->ldv, F->ldv, F->ranks[L - 1],
                                                 tp<T>(F->P), GroupStrides{F->gsy, F->gsy, 256}, bf)));
    for (int p = L - 1; p >= 0; --p) {
      const int q = p + 1;
      const int r = F->ranks[q - 1];
      const int Rp = F->Rp[p];
      const T* segs;
      const int32_t* seg_start;
      hodlr_status s = prod_segments<T>(F, st, fwd_prod_tiles(F, q), q, (int64_t)r * F->Rp[q], tp<T>(F->P),
                                        tp<T>(F->segbuf), &segs, &seg_start);
      if (s) return s;
      const int kp = kpad(r);
      HL("couple_factor", (launch_couple_factor<T>(st, 1 << p, r, kp, Rp, segs, seg_start,
                                                   tp<T>(F->Klu) + F->koff[p], F->Kpiv + F->kvoff[p],
                                                   F->Kperm + F->kvoff[p], tp<T>(F->Kud) + F->kvoff[p],
                                                   tp<T>(F->Kinv) + F->kioff[p], tp<T>(F->W), F->d_info + 1, p, L)));
      if (Rp > 0 && r > 0 && !couple_uses_inverse(r))
        HL("couple_trsm", (launch_block_trsm<T>(st, 0, 1 << p, kp, 2 * r, (int64_t)2 * r * Rp,
                                                tp<T>(F->Klu) + F->koff[p], F->Kperm + F->kvoff[p],
                                                tp<T>(F->Kinv) + F->kioff[p], tp<T>(F->W), 2 * r, Rp)));
      if (p > 0 && r > 0) {
        HL("level_pass",
           (launch_level_pass<T, T, S>(st, F->ntiles[q], F->d_tiles[q], F->tiles_aligned[q], Y, F->ldy, Rp,
                                       Y + (int64_t)Rp * F->ldy, F->ldy, r, tp<T>(F->W), 2 * r, (int64_t)2 * r * Rp, 0,
                                       V + (int64_t)F->Rp[p - 1] * F->ldv, F->ldv, F->ranks[p - 1], tp<T>(F->P),
                                       GroupStrides{F->gsy, F->gsy, 256}, bf)));
      } else if (p > 0) {
        // rank-0 children: no update; products for level p still needed
        HL("level_pass", (launch_level_pass<T, T, S>(st, F->ntiles[q], F->d_tiles[q], F->tiles_aligned[q], Y, F->ldy,
                                                     Rp, (const T*)nullptr, F->ldy, 0, (const T*)nullptr, 0, 0, 0,
                                                     V + (int64_t)F->Rp[p - 1] * F->ldv, F->ldv, F->ranks[p - 1],
                                                     tp<T>(F->P), GroupStrides{F->gsy, F->gsy, 256}, bf)));
      }
    }
  }
  return HODLR_OK;
}

hodlr_status verdict(hodlr_factors* F, hipStream_t st, hodlr_info* info) {
  unsigned long long h[2];
  if (hipMemcpyAsync(h, F->d_info, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess) return HODLR_ERR_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return HODLR_ERR_HIP;
  if (info) {
    info->level = -1;
    info->column = -1;
    info->node = -1;
  }
  F->singular = h[0] != ~0ull || h[1] != ~0ull;
  if (h[0] != ~0ull) {
    if (info) {
      info->level = F->L;
      info->node = (int64_t)(h[0] >> 20);
      info->column = (int32_t)(h[0] & 0xFFFFF);
    }
    return HODLR_ERR_SINGULAR;
  }
  if (h[1] != ~0ull) {
    if (info) {
      info->level = F->L - (int32_t)(h[1] >> 44);
      info->node = (int64_t)((h[1] >> 16) & 0xFFFFFFF);
      info->column = (int32_t)(h[1] & 0xFFFF);
    }
    return HODLR_ERR_SINGULAR;
  }
  return HODLR_OK;
}

hodlr_status dispatch_factor(hodlr_factors* F, hipStream_t st) {
  if (F->compute == HODLR_F64) return run_factor<double, double>(F, st, 0);
  const int bf = F->compute == HODLR_BF16 ? 1 : 0;
  if (F->storage == HODLR_F64) return run_factor<float, double>(F, st, bf);
  return run_factor<float, float>(F, st, bf);
}

// ---- solve-side workspace --------------------------------------------------
// The workspace of stream st (created on first use).
Workspace* get_ws(hodlr_factors* F, hipStream_t st) {
  std::lock_guard<std::mutex> g(F->mu);
  auto it = F->wsmap.find(st);
  if (it != F->wsmap.end()) return it->second.get();
  std::unique_ptr<Workspace> w(new Workspace());
  w->stream = st;
  if (hipEventCreateWithFlags(&w->done, hipEventDisableTiming) != hipSuccess) return nullptr;
  Workspace* p = w.get();
  F->wsmap[st] = std::move(w);
  return p;
}

// Sizes of the solve-side buffers for nrhs columns (elements).
struct WsSizes {
  size_t pmax = 0, segmax = 0, wmax = 0, n = 0, treeN = 0, nrm = 0, ld = 0;
};
WsSizes ws_sizes(const hodlr_factors* F, int nrhs) {
  WsSizes z;
  const int L = F->L;
  for (int p = 1; p <= L; ++p) {
    const size_t elems = (size_t)F->ranks[p - 1] * nrhs;
    for (int q : {fwd_prod_tiles(F, p), adj_prod_tiles(F, p)}) {
      z.pmax = std::max(z.pmax, (size_t)F->ntiles[q] * elems);
      const ProdPlan& pp = F->prods.at({q, p});
      z.segmax = std::max(z.segmax, (pp.buf_items[0] + pp.buf_items[1]) * elems);
    }
  }
  for (int p = 0; p < L; ++p) z.wmax = std::max(z.wmax, (size_t)(int64_t(1) << p) * 2 * F->ranks[p] * nrhs);
  z.n = (size_t)F->n * nrhs;
  z.treeN = std::max<size_t>((((size_t)1 << (L + 1)) - 2) * (size_t)std::max(F->R, 1) * nrhs, 1);
  z.nrm = (size_t)nrhs * (2 * 256 + 8);
  size_t items = F->nleaf;
  for (int p = 0; p < L; ++p)
    if (F->ranks[p] > 0) items += (size_t)1 << p;
  z.ld = 2 * items + 8;  // doubles: logs, then parities (ints) in the second half, then the result
  return z;
}

// Scratch bytes of an unrefined solve with nrhs columns (tile partials, segment
// sums, W, and the compute-type copy of B for FP32 factors), each buffer
// aligned to 256 bytes.
size_t noalloc_bytes(const hodlr_factors* F, int nrhs) {
  const WsSizes z = ws_sizes(F, nrhs);
  const size_t ts = F->tsize;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return al(z.pmax * ts) + al(z.segmax * ts) + al(z.wmax * ts) + (ts == 8 ? 0 : al(z.n * ts));
}

hodlr_status ensure_ws(hodlr_factors* F, Workspace& W, int nrhs) {
  if (nrhs <= W.nrhs) return HODLR_OK;
  // the old buffers may still be read by queued work of this stream
  if (W.nrhs >= 0 && hipStreamSynchronize(W.stream) != hipSuccess) return HODLR_ERR_HIP;
  W.mem.release();
  W.nrhs = -1;
  const size_t ts = F->tsize;
  const WsSizes z = ws_sizes(F, nrhs);
  unsigned char* b;
  hodlr_status s;
  DevMem& M = W.mem;
  if ((s = M.alloc(&b, z.pmax * ts))) return s;
  W.sP = b;
  if ((s = M.alloc(&b, z.segmax * ts))) return s;
  W.sseg = b;
  if ((s = M.alloc(&b, z.wmax * ts))) return s;
  W.sw = b;
  if ((s = M.alloc(&b, z.n * ts))) return s;
  W.sx = b;
  if ((s = M.alloc(&W.rx, z.n))) return s;
  if ((s = M.alloc(&W.rr, z.n))) return s;
  if ((s = M.alloc(&W.tree, z.treeN))) return s;
  if ((s = M.alloc(&W.tree2, z.treeN))) return s;
  if ((s = M.alloc(&W.nrm, z.nrm))) return s;
  if ((s = M.alloc(&W.ld, z.ld))) return s;
  W.nrhs = nrhs;
  return HODLR_OK;
}

// x <- A^{-1} x (trans = 0) or A^{-T} x (trans = 1) in the compute precision, x: N x nrhs, ld N
template <typename T, typename S>
hodlr_status apply_inverse(hodlr_factors* F, Workspace& Wk, hipStream_t st, int trans, int nrhs, T* X, int64_t ldx) {
  const int L = F->L;
  const int64_t N = F->n;
  const T* Y = tp<T>(F->Y);
  const S* V = static_cast<const S*>(F->V);
  T* P = tp<T>(Wk.sP);
  T* w = tp<T>(Wk.sw);
  if (!trans) {
    HL("leaf_solve", (launch_leaf_trsm<T, T>(st, 0, F->nleaf, F->ldl, F->d_off, tp<T>(F->lu), F->lul, F->inplace,
                                             F->perm, tp<T>(F->invl), X, ldx, X, ldx, nrhs)));
    if (L == 0) return HODLR_OK;
    HL("solve_pass", (launch_level_pass<T, T, S>(st, F->ntiles[L], F->d_tiles[L], F->tiles_aligned[L], X, ldx, nrhs, (const T*)nullptr, N,
                                                 0, (const T*)nullptr, 0, 0, 0, V + (int64_t)F->Rp[L - 1] * F->ldv,
                                                 F->ldv, F->ranks[L - 1], P)));
    for (int p = L - 1; p >= 0; --p) {
      const int q = p + 1;
      const int r = F->ranks[q - 1];
      if (r > 0) {
        const T* segs;
        const int32_t* seg_start;
        hodlr_status s = prod_segments<T>(F, st, fwd_prod_tiles(F, q), q, (int64_t)r * nrhs, P, tp<T>(Wk.sseg),
                                          &segs, &seg_start);
        if (s) return s;
        HL("couple_solve", (launch_couple_solve<T>(st, 0, 1 << p, r, kpad(r), nrhs, segs, seg_start,
                                                   tp<T>(F->Klu) + F->koff[p], F->Kperm + F->kvoff[p],
                                                   tp<T>(F->Kud) + F->kvoff[p], w)));
      }
      const int kb = p > 0 ? F->ranks[p - 1] : 0;
      if (r == 0 && kb == 0) continue;
      HL("solve_pass", (launch_level_pass<T, T, S>(st, F->ntiles[q], F->d_tiles[q], F->tiles_aligned[q], X, ldx, nrhs,
                                                   Y + (int64_t)F->Rp[p] * F->ldy, F->ldy, r, w, 2 * r,
                                                   (int64_t)2 * r * nrhs, 0,
                                                   p > 0 ? V + (int64_t)F->Rp[p - 1] * F->ldv : nullptr, F->ldv, kb,
                                                   P, GroupStrides{256, F->gsy, 256})));
    }
    return HODLR_OK;
  }
  // adjoint: top level first, transposed coupling solves, leaves last
  if (L > 0) {
    HL("adjoint_pass", (launch_level_pass<T, S, T>(st, F->ntiles[1], F->d_tiles[1], F->tiles_aligned[1], X, ldx, nrhs, (const S*)nullptr,
                                                   N, 0, (const T*)nullptr, 0, 0, 0, Y, F->ldy, F->ranks[0], P,
                                                   GroupStrides{256, 256, F->gsy})));
    for (int p = 0; p < L; ++p) {
      const int q = p + 1;
      const int r = F->ranks[q - 1];
      if (r > 0) {
        const T* segs;
        const int32_t* seg_start;
        hodlr_status s = prod_segments<T>(F, st, adj_prod_tiles(F, q), q, (int64_t)r * nrhs, P, tp<T>(Wk.sseg),
                                          &segs, &seg_start);
        if (s) return s;
        HL("couple_solve_t", (launch_couple_solve<T>(st, 1, 1 << p, r, kpad(r), nrhs, segs, seg_start,
                                                     tp<T>(F->Klu) + F->koff[p], F->Kperm + F->kvoff[p],
                                                     tp<T>(F->Kud) + F->kvoff[p], w)));
      }
      const int tq = q < L ? q + 1 : L;
      const int kb = q < L ? F->ranks[q] : 0;
      if (r == 0 && kb == 0) continue;
      HL("adjoint_pass", (launch_level_pass<T, S, T>(st, F->ntiles[tq], F->d_tiles[tq], F->tiles_aligned[tq], X, ldx, nrhs,
                                                     V + (int64_t)F->Rp[p] * F->ldv, F->ldv, r, w, 2 * r,
                                                     (int64_t)2 * r * nrhs, tq - q,
                                                     q < L ? Y + (int64_t)F->Rp[q] * F->ldy : nullptr, F->ldy, kb, P,
                                                     GroupStrides{256, 256, F->gsy})));
    }
  }
  HL("leaf_solve_t", (launch_leaf_trsm<T, T>(st, 1, F->nleaf, F->ldl, F->d_off, tp<T>(F->lu), F->lul, F->inplace,
                                             F->perm, tp<T>(F->invl), X, ldx, X, ldx, nrhs)));
  return HODLR_OK;
}

// Y = op(A) X in FP64 from the caller's D, U, V (storage type S); tree: projection workspace
template <typename S>
hodlr_status matvec_impl(hodlr_factors* F, hipStream_t st, int trans, int nrhs, const double* X, int64_t ldx,
                         double* Yo, int64_t ldy, double* tree) {
  const int L = F->L;
  const S* Ua = static_cast<const S*>(trans ? F->V : F->U);
  const S* Vb = static_cast<const S*>(trans ? F->U : F->V);
  const int64_t lda = trans ? F->ldv : F->ldu, ldb = trans ? F->ldu : F->ldv;
  if (L > 0 && F->R > 0) {
    double* leaves = tree + tree_slot(L, 0) * F->R * nrhs;
    HL("mv_project", (launch_level_pass<double, double, S>(st, F->ntiles[L], F->d_tiles[L], F->tiles_aligned[L], const_cast<double*>(X),
                                                           ldx, nrhs, (const double*)nullptr, 0, 0,
                                                           (const double*)nullptr, 0, 0, 0, Vb, ldb, F->R, leaves)));
    for (int l = L - 1; l >= 1; --l)
      HL("mv_tree", launch_tree_sum(st, 1 << l, (int64_t)F->R * nrhs, tree + tree_slot(l + 1, 0) * F->R * nrhs,
                                    tree + tree_slot(l, 0) * F->R * nrhs));
  }
  // every leaf exactly 256 rows (one row per lane of the 4 waves) and every level width a multiple of 4:
  // the kernel needs no masks
  bool full = true;
  for (int a = 0; a < F->nleaf && full; ++a)
    if (F->off[a + 1] - F->off[a] != 256) full = false;
  for (int l = 0; l < L && full; ++l)
    if (F->ranks[l] % 4) full = false;
  HL("mv_apply", (launch_matvec_apply<S>(st, trans, F->nleaf, L, F->d_off, F->d_rpre, F->R,
                                         static_cast<const S*>(F->D), F->ldd, Ua, lda, X, ldx, tree, Yo, ldy, nrhs,
                                         full)));
  return HODLR_OK;
}

hodlr_status matvec_dispatch(hodlr_factors* F, hipStream_t st, int trans, int nrhs, const double* X, int64_t ldx,
                             double* Yo, int64_t ldy, double* tree) {
  if (F->storage == HODLR_F64) return matvec_impl<double>(F, st, trans, nrhs, X, ldx, Yo, ldy, tree);
  return matvec_impl<float>(F, st, trans, nrhs, X, ldx, Yo, ldy, tree);
}

template <typename T>
hodlr_status inverse_dispatch(hodlr_factors* F, Workspace& Wk, hipStream_t st, int trans, int nrhs, T* X,
                              int64_t ldx) {
  // FP64 factors exist only for FP64 storage (checked at factorization)
  if constexpr (sizeof(T) == 8) {
    return apply_inverse<double, double>(F, Wk, st, trans, nrhs, X, ldx);
  } else {
    if (F->storage == HODLR_F64) return apply_inverse<float, double>(F, Wk, st, trans, nrhs, X, ldx);
    return apply_inverse<float, float>(F, Wk, st, trans, nrhs, X, ldx);
  }
}

template <typename T>
hodlr_status solve_impl(hodlr_factors* F, Workspace& Wk, int trans, int nrhs, double* B, int64_t ldb,
                        const hodlr_solve_opts* o, hipStream_t st, hodlr_solve_stats* stt) {
  const int64_t N = F->n;
  if (stt) {
    stt->iters = 0;
    stt->converged = 1;
    stt->relres = 0.0;
  }
  const bool refine = o && o->refine;
  if (!refine) {
    if (sizeof(T) == 8) return inverse_dispatch<T>(F, Wk, st, trans, nrhs, reinterpret_cast<T*>(B), ldb);
    T* x = tp<T>(Wk.sx);
    HL("convert", (launch_convert<T, double>(st, N, nrhs, B, ldb, x, N)));
    hodlr_status s = inverse_dispatch<T>(F, Wk, st, trans, nrhs, x, N);
    if (s) return s;
    HL("convert", (launch_convert<double, T>(st, N, nrhs, x, N, B, ldb)));
    return HODLR_OK;
  }
  // FP64 iterative refinement
  const double tol = o->tol > 0 ? o->tol : 1e-10;
  const int max_iter = o->max_iter > 0 ? o->max_iter : 30;
  double* part = Wk.nrm;
  double* b2 = part + (size_t)nrhs * 512;
  double* r2 = b2 + nrhs;
  double* rinf = r2 + nrhs;
  double* x = Wk.rx;
  double* r = Wk.rr;
  T* t = tp<T>(Wk.sx);
  hodlr_status s;
  HL("norms", launch_colnorms(st, N, nrhs, B, ldb, part, b2, rinf));
  if (hipMemsetAsync(x, 0, (size_t)N * nrhs * 8, st) != hipSuccess) return HODLR_ERR_HIP;
  if (hipMemcpy2DAsync(r, N * 8, B, ldb * 8, N * 8, nrhs, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return HODLR_ERR_HIP;
  std::vector<double> hb(nrhs), hr(nrhs);
  if (hipMemcpyAsync(hb.data(), b2, nrhs * 8, hipMemcpyDeviceToHost, st) != hipSuccess) return HODLR_ERR_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return HODLR_ERR_HIP;
  double prev = INFINITY, res = 0.0;
  int grow = 0, it = 0;
  for (int j = 0; j < nrhs; ++j) res = std::max(res, 1.0);  // r = b initially
  if (nrhs == 0) res = 0.0;
  while (res > tol && it < max_iter) {
    HL("refine_scale", (launch_scale_down<T>(st, N, nrhs, r, N, rinf, t, N)));
    s = inverse_dispatch<T>(F, Wk, st, trans, nrhs, t, N);
    if (s) return s;
    HL("refine_axpy", (launch_axpy_up<T>(st, N, nrhs, t, N, rinf, x, N)));
    s = matvec_dispatch(F, st, trans, nrhs, x, N, r, N, Wk.tree);
    if (s) return s;
    HL("refine_residual", launch_residual(st, N, nrhs, B, ldb, r, N));
    HL("norms", launch_colnorms(st, N, nrhs, r, N, part, r2, rinf));
    if (hipMemcpyAsync(hr.data(), r2, nrhs * 8, hipMemcpyDeviceToHost, st) != hipSuccess) return HODLR_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return HODLR_ERR_HIP;
    ++it;
    res = 0.0;
    for (int j = 0; j < nrhs; ++j) {
      const double rj = hb[j] > 0 ? hr[j] / hb[j] : hr[j];
      res = std::isfinite(rj) ? std::max(res, rj) : INFINITY;  // a NaN/Inf residual is divergence
    }
    grow = (res > prev) ? grow + 1 : 0;
    prev = res;
    if (grow >= 2) break;
  }
  if (hipMemcpy2DAsync(B, ldb * 8, x, N * 8, N * 8, nrhs, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return HODLR_ERR_HIP;
  if (stt) {
    stt->iters = it;
    stt->relres = res;
    stt->converged = res <= tol;
  }
  return res <= tol ? HODLR_OK : HODLR_ERR_NOT_CONVERGED;
}

// One call on stream st with that stream's workspace: waits (on the device)
// for the factorization, runs fn, and records the workspace's done event.
template <typename Fn>
hodlr_status on_stream(hodlr_factors* F, hipStream_t st, int nrhs, Fn fn) {
  Workspace* W = get_ws(F, st);
  if (!W) return HODLR_ERR_HIP;
  std::lock_guard<std::mutex> g(W->mu);
  hodlr_status s = ensure_ws(F, *W, nrhs);
  if (s) return s;
  if (hipStreamWaitEvent(st, F->ready, 0) != hipSuccess) return HODLR_ERR_HIP;
  s = fn(*W);
  if (hipEventRecord(W->done, st) != hipSuccess && s >= 0) s = HODLR_ERR_HIP;
  return s;
}

hodlr_status solve_common(const hodlr_factors* Fc, int trans, int64_t nrhs, double* B, int64_t ldb,
                          const hodlr_solve_opts* o, void* stream, hodlr_solve_stats* stt) {
  hodlr_factors* F = const_cast<hodlr_factors*>(Fc);
  if (!F || nrhs < 0 || nrhs > 65535) return HODLR_ERR_ARG;
  if (F->cplx) ldb *= 2;  // complex columns: interleaved (re, im), the embedded real vector
  if (nrhs > 0 && (!B || ldb < F->n)) return HODLR_ERR_ARG;
  if (o && o->refine && F->inplace) return HODLR_ERR_ARG;  // the residual needs the original D and U
  if (nrhs == 0) return HODLR_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return on_stream(F, st, (int)nrhs, [&](Workspace& W) {
    if (F->compute == HODLR_F64) return solve_impl<double>(F, W, trans, (int)nrhs, B, ldb, o, st, stt);
    return solve_impl<float>(F, W, trans, (int)nrhs, B, ldb, o, st, stt);
  });
}

hodlr_status setup(hodlr_factors* F, const hodlr_matrix* A, hodlr_dtype compute, int32_t flags) {
  std::vector<int64_t> off;
  std::vector<int> ranks;
  int m_max = 0;
  hodlr_status s = validate(A, off, ranks, m_max);
  if (s) return s;
  if (flags & ~HODLR_INPLACE) return HODLR_ERR_ARG;
  if (compute != HODLR_F64 && compute != HODLR_F32 && compute != HODLR_BF16) return HODLR_ERR_ARG;
  if (compute == HODLR_F64 && A->dtype != HODLR_F64) return HODLR_ERR_UNSUPPORTED;
  if (flags & HODLR_INPLACE) {
    // the factors take the caller's storage: same element type, and every leaf a
    // whole number of 16-row blocks (no padded block may reach into a neighbour)
    if ((compute == HODLR_F64) != (A->dtype == HODLR_F64)) return HODLR_ERR_UNSUPPORTED;
    for (size_t i = 0; i + 1 < off.size(); ++i)
      if ((off[i + 1] - off[i]) % 16) return HODLR_ERR_UNSUPPORTED;
  }
  F->inplace = (flags & HODLR_INPLACE) ? 1 : 0;
  F->n = A->n;
  F->L = A->levels;
  F->nleaf = 1 << F->L;
  F->m_max = m_max;
  F->ldl = (m_max + 15) & ~15;
  F->off = off;
  F->ranks = ranks;
  F->Rp.assign(F->L + 1, 0);
  for (int l = 1; l <= F->L; ++l) F->Rp[l] = F->Rp[l - 1] + ranks[l - 1];
  F->R = F->Rp[F->L];
  F->storage = A->dtype;
  F->compute = compute;
  F->tsize = tsz(compute);
  F->D = A->D;
  F->U = A->U;
  F->V = A->V;
  F->ldd = A->ldd;
  F->ldu = A->ldu;
  F->ldv = A->ldv;
  return HODLR_OK;
}

hodlr_status grad_impl(hodlr_factors* F, Workspace& Wk, hipStream_t st, int64_t nrhs, const double* X, int64_t ldx,
                       const double* Lam, int64_t ldl, void* dD, void* dU, void* dV);

// Complex matrix A (dtype HODLR_C128) as the real HODLR matrix emb(A): same
// tree, leaf offsets and ranks doubled, D~ = emb(D) (2N x 2 m_max), U~ =
// emb(U), V~ = emb(V) (2N x 2R), all with leading dimension 2N.  Validates A
// and writes the embedded copies into D, U, V (allocated in M when null).
struct Embedded {
  hodlr_matrix E{};
  std::vector<int64_t> off;
  std::vector<int32_t> ranks;
};
hodlr_status embed_complex(const hodlr_matrix* A, hipStream_t st, DevMem& M, Embedded& X, double* D, double* U,
                           double* V) {
  if (!A || A->dtype != HODLR_C128) return HODLR_ERR_ARG;
  hodlr_matrix Ar = *A;
  Ar.dtype = HODLR_F64;
  std::vector<int64_t> off;
  std::vector<int> ranks;
  int m_max = 0;
  hodlr_status s = validate(&Ar, off, ranks, m_max);
  if (s) return s;
  if (2 * m_max > HODLR_MAX_LEAF) return HODLR_ERR_UNSUPPORTED;
  int R = 0;
  for (int r : ranks) {
    if (2 * r > HODLR_MAX_RANK) return HODLR_ERR_UNSUPPORTED;
    R += r;
  }
  if (A->n > (int64_t(1) << 40)) return HODLR_ERR_UNSUPPORTED;
  const int64_t n2 = 2 * A->n;
  if (!D && (s = M.alloc(&D, (size_t)n2 * 2 * m_max))) return s;
  if (R > 0 && !U && (s = M.alloc(&U, (size_t)n2 * 2 * R))) return s;
  if (R > 0 && !V && (s = M.alloc(&V, (size_t)n2 * 2 * R))) return s;
  // the caller's D beyond each leaf's width is embedded too and never read
  HL("embed", launch_embed_cols(st, A->n, m_max, static_cast<const double*>(A->D), A->ldd, D, n2));
  if (R > 0) {
    HL("embed", launch_embed_cols(st, A->n, R, static_cast<const double*>(A->U), A->ldu, U, n2));
    HL("embed", launch_embed_cols(st, A->n, R, static_cast<const double*>(A->V), A->ldv, V, n2));
  }
  X.off.resize(off.size());
  for (size_t i = 0; i < off.size(); ++i) X.off[i] = 2 * off[i];
  X.ranks.resize(ranks.size());
  for (size_t i = 0; i < ranks.size(); ++i) X.ranks[i] = 2 * ranks[i];
  X.E = hodlr_matrix{n2, A->levels, X.off.data(), X.ranks.empty() ? nullptr : X.ranks.data(), HODLR_F64, D, n2,
                     R > 0 ? U : nullptr, n2, R > 0 ? V : nullptr, n2};
  return HODLR_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

hodlr_status hodlr_factor(const hodlr_matrix* A, hodlr_dtype compute, int32_t flags, void* stream,
                          hodlr_factors** out, hodlr_info* info) {
  if (!out) return HODLR_ERR_ARG;
  *out = nullptr;
  if (A && A->dtype == HODLR_C128) {
    // factor the real embedding, which the factorization then owns
    if (flags & HODLR_INPLACE) return HODLR_ERR_UNSUPPORTED;
    hipStream_t st = static_cast<hipStream_t>(stream);
    DevMem M;
    Embedded X;
    hodlr_status s = embed_complex(A, st, M, X, nullptr, nullptr, nullptr);
    if (s == HODLR_OK) s = hodlr_factor(&X.E, compute, 0, stream, out, info);
    if (*out) {
      (*out)->cplx = 1;
      (*out)->emb = std::move(M);
    } else {
      hipStreamSynchronize(st);
      M.release();
    }
    return s;
  }
  hodlr_factors* F = new hodlr_factors();
  hodlr_status s = setup(F, A, compute, flags);
  if (s == HODLR_OK) s = allocate_factors(F);
  if (s != HODLR_OK) {
    F->mem.release();
    if (F->ready) hipEventDestroy(F->ready);
    if (F->na_done) hipEventDestroy(F->na_done);
    delete F;
    return s;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  s = dispatch_factor(F, st);
  if (s == HODLR_OK && hipEventRecord(F->ready, st) != hipSuccess) s = HODLR_ERR_HIP;
  if (s == HODLR_OK) s = verdict(F, st, info);
  if (s < 0) {
    hipStreamSynchronize(st);
    F->mem.release();
    hipEventDestroy(F->ready);
    hipEventDestroy(F->na_done);
    delete F;
    return s;
  }
  *out = F;
  return s;
}

hodlr_status hodlr_refactor(hodlr_factors* F, const hodlr_matrix* A, void* stream, hodlr_info* info) {
  if (!F || !A) return HODLR_ERR_ARG;
  if ((A->dtype == HODLR_C128) != (F->cplx != 0)) return HODLR_ERR_ARG;
  std::vector<int64_t> off;
  std::vector<int> ranks;
  int m_max = 0;
  hodlr_status s;
  if (F->cplx) {
    // same tree and ranks; the leading dimensions of the caller's arrays may change
    hodlr_matrix Ar = *A;
    Ar.dtype = HODLR_F64;
    if ((s = validate(&Ar, off, ranks, m_max))) return s;
    for (auto& o : off) o *= 2;
    for (auto& r : ranks) r *= 2;
    if (2 * A->n != F->n || A->levels != F->L || off != F->off || ranks != F->ranks) return HODLR_ERR_ARG;
  } else {
    if ((s = validate(A, off, ranks, m_max))) return s;
    if (A->n != F->n || A->levels != F->L || off != F->off || ranks != F->ranks || A->dtype != F->storage ||
        A->ldd != F->ldd || A->ldu != F->ldu || A->ldv != F->ldv)
      return HODLR_ERR_ARG;
  }
  std::lock_guard<std::mutex> g(F->mu);
  hipStream_t st = static_cast<hipStream_t>(stream);
  // no call on another stream may still read the old factors: hold every
  // workspace and make this stream wait for the work each one last recorded
  std::vector<std::unique_lock<std::mutex>> held;
  for (auto& kv : F->wsmap) {
    held.emplace_back(kv.second->mu);
    if (hipStreamWaitEvent(st, kv.second->done, 0) != hipSuccess) return HODLR_ERR_HIP;
  }
  std::lock_guard<std::mutex> gna(F->na_mu);
  if (hipStreamWaitEvent(st, F->na_done, 0) != hipSuccess) return HODLR_ERR_HIP;
  if (F->cplx) {
    // new values into the embedded copies the factorization owns
    DevMem none;
    Embedded X;
    if ((s = embed_complex(A, st, none, X, static_cast<double*>(const_cast<void*>(F->D)),
                           static_cast<double*>(const_cast<void*>(F->U)), static_cast<double*>(const_cast<void*>(F->V)))))
      return s;
    s = dispatch_factor(F, st);
    if (s == HODLR_OK && hipEventRecord(F->ready, st) != hipSuccess) s = HODLR_ERR_HIP;
    if (s == HODLR_OK) s = verdict(F, st, info);
    return s;
  }
  F->D = A->D;
  F->U = A->U;
  F->V = A->V;
  if (F->inplace) {
    F->lu = const_cast<void*>(F->D);
    F->Y = const_cast<void*>(F->U);
  }
  s = dispatch_factor(F, st);
  if (s == HODLR_OK && hipEventRecord(F->ready, st) != hipSuccess) s = HODLR_ERR_HIP;
  if (s == HODLR_OK) s = verdict(F, st, info);
  return s;
}

hodlr_status hodlr_solve(const hodlr_factors* F, int64_t nrhs, double* B, int64_t ldb, const hodlr_solve_opts* o,
                         void* stream, hodlr_solve_stats* st) {
  return solve_common(F, 0, nrhs, B, ldb, o, stream, st);
}

hodlr_status hodlr_solve_adjoint(const hodlr_factors* F, int64_t nrhs, double* B, int64_t ldb,
                                 const hodlr_solve_opts* o, void* stream, hodlr_solve_stats* st) {
  return solve_common(F, 1, nrhs, B, ldb, o, stream, st);
}

size_t hodlr_solve_noalloc_bytes(const hodlr_factors* F, int64_t nrhs) {
  if (!F || nrhs < 0 || nrhs > 65535) return 0;
  return noalloc_bytes(F, (int)nrhs);
}

hodlr_status hodlr_solve_noalloc(const hodlr_factors* Fc, int32_t trans, int64_t nrhs, double* B, int64_t ldb,
                                 void* stream) {
  hodlr_factors* F = const_cast<hodlr_factors*>(Fc);
  if (!F || (trans != 0 && trans != 1) || nrhs < 0 || nrhs > 65535) return HODLR_ERR_ARG;
  if (F->cplx) ldb *= 2;
  if (nrhs > 0 && (!B || ldb < F->n)) return HODLR_ERR_ARG;
  if (nrhs == 0) return HODLR_OK;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return HODLR_ERR_HIP;
  if (dev != F->device) return HODLR_ERR_ARG;
  const size_t need = noalloc_bytes(F, (int)nrhs);
  if (need > scratch_capacity()) return HODLR_ERR_ARG;
  void* base = nullptr;
  if (scratch_device_ptr(&base) != hipSuccess) return HODLR_ERR_HIP;
  // the solve-side buffers carved out of this device's scratch (every byte
  // the solve reads there is written earlier in the same call)
  Workspace W;
  unsigned char* p = static_cast<unsigned char*>(base);
  const WsSizes z = ws_sizes(F, (int)nrhs);
  const size_t ts = F->tsize;
  auto take = [&](size_t bytes) {
    void* q = p;
    p += (bytes + 255) & ~size_t(255);
    return q;
  };
  W.sP = take(z.pmax * ts);
  W.sseg = take(z.segmax * ts);
  W.sw = take(z.wmax * ts);
  W.sx = ts == 8 ? nullptr : take(z.n * ts);
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> g(F->na_mu);
  if (hipStreamWaitEvent(st, F->ready, 0) != hipSuccess) return HODLR_ERR_HIP;
  hodlr_status s = F->compute == HODLR_F64 ? solve_impl<double>(F, W, trans, (int)nrhs, B, ldb, nullptr, st, nullptr)
                                           : solve_impl<float>(F, W, trans, (int)nrhs, B, ldb, nullptr, st, nullptr);
  if (hipEventRecord(F->na_done, st) != hipSuccess && s >= 0) s = HODLR_ERR_HIP;
  return s;
}

hodlr_status hodlr_matvec(const hodlr_matrix* A, int32_t trans, int64_t nrhs, const double* X, int64_t ldx, double* Yo,
                          int64_t ldy, void* stream) {
  if (nrhs < 0 || nrhs > 65535) return HODLR_ERR_ARG;
  if (A && A->dtype == HODLR_C128) {
    if (nrhs > 0 && (!X || !Yo || ldx < A->n || ldy < A->n)) return HODLR_ERR_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    DevMem M;
    Embedded E;
    hodlr_status s = embed_complex(A, st, M, E, nullptr, nullptr, nullptr);
    if (s == HODLR_OK) s = hodlr_matvec(&E.E, trans, nrhs, X, 2 * ldx, Yo, 2 * ldy, stream);
    hipStreamSynchronize(st);
    M.release();
    return s;
  }
  hodlr_factors F;
  std::vector<int64_t> off;
  std::vector<int> ranks;
  int m_max = 0;
  hodlr_status s = validate(A, off, ranks, m_max);
  if (s) return s;
  if (nrhs == 0) return HODLR_OK;
  if (!X || !Yo || ldx < A->n || ldy < A->n) return HODLR_ERR_ARG;
  s = setup(&F, A, A->dtype == HODLR_F64 ? HODLR_F64 : HODLR_F32, 0);
  if (s) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = F.mem.alloc(&F.d_off, F.off.size()))) return s;
  std::vector<int32_t> rp(F.Rp.begin(), F.Rp.end());
  s = F.mem.alloc(&F.d_rpre, rp.size());
  if (!s && hipMemcpy(F.d_off, F.off.data(), F.off.size() * 8, hipMemcpyHostToDevice) != hipSuccess) s = HODLR_ERR_HIP;
  if (!s && hipMemcpy(F.d_rpre, rp.data(), rp.size() * 4, hipMemcpyHostToDevice) != hipSuccess) s = HODLR_ERR_HIP;
  if (!s) s = plan(&F);
  double* tree = nullptr;
  const size_t treeN = (((size_t)1 << (F.L + 1)) - 2) * (size_t)std::max(F.R, 1) * nrhs;
  if (!s) s = F.mem.alloc(&tree, std::max<size_t>(treeN, 1));
  if (!s) s = matvec_dispatch(&F, st, trans ? 1 : 0, (int)nrhs, X, ldx, Yo, ldy, tree);
  hipStreamSynchronize(st);
  F.mem.release();
  return s;
}

hodlr_status hodlr_grad(const hodlr_factors* Fc, int64_t nrhs, const double* X, int64_t ldx, const double* Lam,
                        int64_t ldl, void* dD, void* dU, void* dV, void* stream) {
  hodlr_factors* F = const_cast<hodlr_factors*>(Fc);
  if (!F || nrhs < 1 || nrhs > 65535 || !X || !Lam || ldx < F->n || ldl < F->n || !dD) return HODLR_ERR_ARG;
  if (F->R > 0 && (!dU || !dV)) return HODLR_ERR_ARG;
  if (F->inplace) return HODLR_ERR_ARG;  // the gradients need the original U and V
  if (F->cplx) return HODLR_ERR_UNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return on_stream(F, st, (int)nrhs, [&](Workspace& Wk) { return grad_impl(F, Wk, st, nrhs, X, ldx, Lam, ldl, dD, dU, dV); });
}

}  // extern "C"

namespace {
hodlr_status grad_impl(hodlr_factors* F, Workspace& Wk, hipStream_t st, int64_t nrhs, const double* X, int64_t ldx,
                       const double* Lam, int64_t ldl, void* dD, void* dU, void* dV) {
  hodlr_status s;
  const int L = F->L;
  const int n = (int)nrhs;
  auto project = [&](const void* Mv, int64_t ldm, const double* Xin, int64_t ldxin, double* tree) -> hodlr_status {
    if (L == 0 || F->R == 0) return HODLR_OK;
    double* leaves = tree + tree_slot(L, 0) * F->R * n;
    if (F->storage == HODLR_F64)
      HL("grad_project", (launch_level_pass<double, double, double>(
                             st, F->ntiles[L], F->d_tiles[L], F->tiles_aligned[L], const_cast<double*>(Xin), ldxin, n, (const double*)nullptr,
                             0, 0, (const double*)nullptr, 0, 0, 0, static_cast<const double*>(Mv), ldm, F->R, leaves)));
    else
      HL("grad_project", (launch_level_pass<double, double, float>(
                             st, F->ntiles[L], F->d_tiles[L], F->tiles_aligned[L], const_cast<double*>(Xin), ldxin, n, (const double*)nullptr,
                             0, 0, (const double*)nullptr, 0, 0, 0, static_cast<const float*>(Mv), ldm, F->R, leaves)));
    for (int l = L - 1; l >= 1; --l)
      HL("grad_tree", launch_tree_sum(st, 1 << l, (int64_t)F->R * n, tree + tree_slot(l + 1, 0) * F->R * n,
                                      tree + tree_slot(l, 0) * F->R * n));
    return HODLR_OK;
  };
  if ((s = project(F->V, F->ldv, X, ldx, Wk.tree))) return s;     // V^T X node sums
  if ((s = project(F->U, F->ldu, Lam, ldl, Wk.tree2))) return s;  // U^T Lambda node sums
  if (F->storage == HODLR_F64) {
    HL("grad_leaf", (launch_grad_leaf<double>(st, F->nleaf, F->m_max, F->d_off, n, X, ldx, Lam, ldl,
                                              static_cast<double*>(dD), F->ldd)));
    if (F->R > 0 && L > 0) {
      HL("grad_gen", (launch_grad_gen<double>(st, F->nleaf, L, F->d_off, F->d_rpre, F->R, n, Lam, ldl, Wk.tree,
                                              static_cast<double*>(dU), F->ldu)));
      HL("grad_gen", (launch_grad_gen<double>(st, F->nleaf, L, F->d_off, F->d_rpre, F->R, n, X, ldx, Wk.tree2,
                                              static_cast<double*>(dV), F->ldv)));
    }
  } else {
    HL("grad_leaf", (launch_grad_leaf<float>(st, F->nleaf, F->m_max, F->d_off, n, X, ldx, Lam, ldl,
                                             static_cast<float*>(dD), F->ldd)));
    if (F->R > 0 && L > 0) {
      HL("grad_gen", (launch_grad_gen<float>(st, F->nleaf, L, F->d_off, F->d_rpre, F->R, n, Lam, ldl, Wk.tree,
                                             static_cast<float*>(dU), F->ldu)));
      HL("grad_gen", (launch_grad_gen<float>(st, F->nleaf, L, F->d_off, F->d_rpre, F->R, n, X, ldx, Wk.tree2,
                                             static_cast<float*>(dV), F->ldv)));
    }
  }
  return HODLR_OK;
}
}  // namespace

extern "C" {

hodlr_status hodlr_factors_y(const hodlr_factors* F, double* Yo, int64_t ldy, void* stream) {
  if (!F || (F->R > 0 && (!Yo || ldy < (F->cplx ? F->n / 2 : F->n)))) return HODLR_ERR_ARG;
  if (F->R == 0) return HODLR_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  DevMem M;
  double* Yr = Yo;
  int64_t ldr = ldy;
  if (F->cplx) {  // the embedded Y first, then the complex Y from it
    if (M.alloc(&Yr, (size_t)F->n * F->R)) return HODLR_ERR_ALLOC;
    ldr = F->n;
  }
  auto convert = [&]() -> hodlr_status {
    if (F->compute == HODLR_F64)
      HL("convert", (launch_convert<double, double>(st, F->n, F->R, static_cast<const double*>(F->Y), F->ldy, Yr, ldr,
                                                    F->gsy)));
    else
      HL("convert", (launch_convert<double, float>(st, F->n, F->R, static_cast<const float*>(F->Y), F->ldy, Yr, ldr,
                                                   F->gsy)));
    // Y~ = emb(Y) (a product of embeddings is the embedding of the product): the
    // complex Y from the first column of each 2 x 2 block
    if (F->cplx) HL("embed", launch_deembed_cols(st, F->n / 2, F->R / 2, Yr, F->n, Yo, ldy));
    return HODLR_OK;
  };
  hodlr_status s = convert();
  if (F->cplx) {
    hipStreamSynchronize(st);
    M.release();
  }
  return s;
}

hodlr_status hodlr_logdet(const hodlr_factors* Fc, double* sign, double* logabs, void* stream) {
  hodlr_factors* F = const_cast<hodlr_factors*>(Fc);
  if (!F || !sign || !logabs) return HODLR_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  LogdetLevels lv;
  for (int p = 0; p < F->L; ++p) {
    const int r = F->ranks[p];
    if (r == 0) continue;
    lv.count[lv.n] = 1 << p;
    lv.r[lv.n] = r;
    lv.kp[lv.n] = kpad(r);
    lv.kvoff[lv.n] = F->kvoff[p];
    ++lv.n;
  }
  if (F->singular) {  // an exactly zero pivot: det A = 0 (later factors are not meaningful)
    *sign = 0.0;
    *logabs = -INFINITY;
    return HODLR_OK;
  }
  double res[2] = {0.0, 0.0};
  hodlr_status s = on_stream(F, st, 1, [&](Workspace& W) -> hodlr_status {
    size_t items = F->nleaf;
    for (int p = 0; p < lv.n; ++p) items += lv.count[p];
    double* logs = W.ld;
    int* par = reinterpret_cast<int*>(W.ld + items);
    double* out = W.ld + 2 * items;
    if (F->compute == HODLR_F64)
      HL("logdet", (launch_logdet<double>(st, F->nleaf, F->ldl, F->d_off, tp<double>(F->udinv), F->piv,
                                          tp<double>(F->Kud), F->Kpiv, lv, logs, par, out)));
    else
      HL("logdet", (launch_logdet<float>(st, F->nleaf, F->ldl, F->d_off, tp<float>(F->udinv), F->piv,
                                         tp<float>(F->Kud), F->Kpiv, lv, logs, par, out)));
    if (hipMemcpyAsync(res, out, sizeof(res), hipMemcpyDeviceToHost, st) != hipSuccess) return HODLR_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return HODLR_ERR_HIP;
    return HODLR_OK;
  });
  if (s) return s;
  *logabs = res[0];
  *sign = std::isinf(res[0]) && res[0] < 0 ? 0.0 : res[1];
  if (F->cplx) {
    // det emb(A) = |det A|^2 >= 0: log|det A| is half of it; the phase of det A
    // is not available (sign 1, or 0 when singular)
    *logabs *= 0.5;
    *sign = *sign == 0.0 ? 0.0 : 1.0;
  }
  return HODLR_OK;
}

}  // extern "C"

namespace {
// K^{-1} diagonal blocks P_a of every level, FP64, Pd at pdoff[l] + a r_l^2
template <typename T>
hodlr_status logdet_pblocks(hodlr_factors* F, hipStream_t st, DevMem& M, double* Pd,
                            const std::vector<int64_t>& pdoff) {
  for (int p = 0; p < F->L; ++p) {
    const int r = F->ranks[p];
    if (r == 0) continue;
    const int np = 1 << p, n2 = 2 * r, kp = kpad(r);
    double* Pl = Pd + pdoff[p + 1];
    if (couple_uses_inverse(r)) {  // K^{-1} is stored (n2 x n2 per parent)
      HL("logdet_grad", launch_pblocks<T>(st, np, r, tp<T>(F->Klu) + F->koff[p], n2, (int64_t)n2 * n2, Pl));
    } else {  // K^{-1} = K^{-1} I by the block solver on the stored LU
      T* X = nullptr;
      hodlr_status s = M.alloc(&X, (size_t)np * n2 * n2);
      if (s) return s;
      HL("logdet_grad", launch_identity_blocks<T>(st, np, n2, X));
      HL("logdet_grad", launch_block_trsm<T>(st, 0, np, kp, n2, n2, tp<T>(F->Klu) + F->koff[p], F->Kperm + F->kvoff[p],
                                              tp<T>(F->Kinv) + F->kioff[p], X, (int64_t)np * n2, n2));
      HL("logdet_grad", launch_pblocks<T>(st, np, r, X, (int64_t)np * n2, n2, Pl));
    }
  }
  return HODLR_OK;
}

template <typename T, typename S>
hodlr_status logdet_grad_impl(hodlr_factors* F, hipStream_t st, DevMem& M, void* dDv, void* dUv, void* dVv) {
  const int L = F->L, R = F->R;
  const int64_t N = F->n;
  hodlr_status s;
  S* dD = static_cast<S*>(dDv);
  S* dU = static_cast<S*>(dUv);
  S* dV = static_cast<S*>(dVv);
  // D^{-T} on the leaf blocks: the adjoint leaf solve of the identity
  T* E = nullptr;
  double* E64 = nullptr;
  if ((s = M.alloc(&E, (size_t)N * F->m_max)) || (s = M.alloc(&E64, (size_t)N * F->m_max))) return s;
  HL("logdet_grad", launch_identity_leaves<T>(st, F->nleaf, F->m_max, F->d_off, E, N));
  HL("logdet_grad", (launch_leaf_trsm<T, T>(st, 1, F->nleaf, F->ldl, F->d_off, tp<T>(F->lu), F->lul, F->inplace,
                                             F->perm, tp<T>(F->invl), E, N, E, N, F->m_max)));
  HL("logdet_grad", (launch_convert<double, T>(st, N, F->m_max, E, N, E64, N)));
  if (L == 0 || R == 0) {
    HL("logdet_grad", launch_grad_leaf<S>(st, F->nleaf, F->m_max, F->d_off, 0, E64, N, E64, N, dD, F->ldd, E64, N));
    return HODLR_OK;
  }
  // Y_big of A^T (D^T, generators exchanged): its level-l block at I_a is A_a^{-T} V_a
  S* Dt = nullptr;
  if ((s = M.alloc(&Dt, (size_t)N * F->m_max))) return s;
  HL("logdet_grad", launch_transpose_leaves<S>(st, F->nleaf, F->m_max, F->d_off, static_cast<const S*>(F->D), F->ldd,
                                                Dt, N));
  std::vector<int32_t> rk(F->ranks.begin(), F->ranks.end());
  hodlr_matrix At{};
  At.n = N;
  At.levels = L;
  At.leaf_offsets = F->off.data();
  At.ranks = rk.data();
  At.dtype = F->storage;
  At.D = Dt;
  At.ldd = N;
  At.U = F->V;
  At.ldu = F->ldv;
  At.V = F->U;
  At.ldv = F->ldu;
  hodlr_factors* FT = nullptr;
  s = hodlr_factor(&At, F->compute, 0, st, &FT, nullptr);
  if (s) {
    if (FT) hodlr_destroy(FT);
    return s < 0 ? s : HODLR_ERR_SINGULAR;
  }
  struct Guard {
    hodlr_factors* f;
    ~Guard() { hodlr_destroy(f); }
  } guard{FT};
  double *Y64 = nullptr, *Yt64 = nullptr, *Lam = nullptr, *YP = nullptr, *Pd = nullptr, *tV = nullptr, *tU = nullptr;
  int64_t* d_pdoff = nullptr;
  std::vector<int64_t> pdoff(L + 2, 0);
  for (int l = 1; l <= L; ++l) pdoff[l + 1] = pdoff[l] + ((int64_t)1 << l) * F->ranks[l - 1] * F->ranks[l - 1];
  const size_t nr = (size_t)N * R;
  const size_t treeN = (((size_t)1 << (L + 1)) - 2) * (size_t)R * R;
  if ((s = M.alloc(&Y64, nr)) || (s = M.alloc(&Yt64, nr)) || (s = M.alloc(&Lam, nr)) || (s = M.alloc(&YP, nr)) ||
      (s = M.alloc(&Pd, std::max<size_t>(pdoff[L + 1], 1))) || (s = M.alloc(&d_pdoff, pdoff.size())) ||
      (s = M.alloc(&tV, treeN)) || (s = M.alloc(&tU, treeN)))
    return s;
  if (hipMemcpyAsync(d_pdoff, pdoff.data(), pdoff.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess)
    return HODLR_ERR_HIP;
  HL("logdet_grad", (launch_convert<double, T>(st, N, R, tp<T>(F->Y), F->ldy, Y64, N, F->gsy)));
  HL("logdet_grad", (launch_convert<double, T>(st, N, R, tp<T>(FT->Y), FT->ldy, Yt64, N, FT->gsy)));
  if ((s = logdet_pblocks<T>(F, st, M, Pd, pdoff))) return s;
  // Lam(I_a, c_l) = (A_a^{-T} V_a) P_a^T; YP(I_a, c_l) = Y_a P_a
  HL("logdet_grad", launch_node_mix(st, N, L, R, F->d_off, F->d_rpre, d_pdoff, Pd, 1, Yt64, Lam));
  HL("logdet_grad", launch_node_mix(st, N, L, R, F->d_off, F->d_rpre, d_pdoff, Pd, 0, Y64, YP));
  // dD = D^{-T} - Lam Y^T on the leaf blocks
  HL("logdet_grad", launch_grad_leaf<S>(st, F->nleaf, F->m_max, F->d_off, R, Y64, N, Lam, N, dD, F->ldd, E64, N));
  // projection trees V^T Y and U^T Lam (per node, all columns)
  auto project = [&](const void* Mv, int64_t ldm, const double* Xin, double* tree) -> hodlr_status {
    double* leaves = tree + tree_slot(L, 0) * (int64_t)R * R;
    HL("logdet_grad", (launch_level_pass<double, double, S>(st, F->ntiles[L], F->d_tiles[L], F->tiles_aligned[L],
                                                            const_cast<double*>(Xin), N, R, (const double*)nullptr, 0,
                                                            0, (const double*)nullptr, 0, 0, 0,
                                                            static_cast<const S*>(Mv), ldm, R, leaves)));
    for (int l = L - 1; l >= 1; --l)
      HL("logdet_grad", launch_tree_sum(st, 1 << l, (int64_t)R * R, tree + tree_slot(l + 1, 0) * (int64_t)R * R,
                                        tree + tree_slot(l, 0) * (int64_t)R * R));
    return HODLR_OK;
  };
  if ((s = project(F->V, F->ldv, Y64, tV))) return s;
  if ((s = project(F->U, F->ldu, Lam, tU))) return s;
  HL("logdet_grad", launch_grad_gen<S>(st, F->nleaf, L, F->d_off, F->d_rpre, R, R, Lam, N, tV, dU, F->ldu, Lam, N, 1));
  HL("logdet_grad", launch_grad_gen<S>(st, F->nleaf, L, F->d_off, F->d_rpre, R, R, Y64, N, tU, dV, F->ldv, YP, N, 1));
  return HODLR_OK;
}
}  // namespace

extern "C" {

hodlr_status hodlr_logdet_grad(const hodlr_factors* Fc, void* dD, void* dU, void* dV, void* stream) {
  hodlr_factors* F = const_cast<hodlr_factors*>(Fc);
  if (!F || !dD || (F->R > 0 && (!dU || !dV))) return HODLR_ERR_ARG;
  if (F->inplace) return HODLR_ERR_ARG;  // needs the original D, U, V
  if (F->cplx) return HODLR_ERR_UNSUPPORTED;
  if (F->singular) return HODLR_ERR_SINGULAR;  // log|det A| is -inf: no gradient
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipStreamWaitEvent(st, F->ready, 0) != hipSuccess) return HODLR_ERR_HIP;
  DevMem M;
  hodlr_status s;
  if (F->compute == HODLR_F64)
    s = logdet_grad_impl<double, double>(F, st, M, dD, dU, dV);
  else if (F->storage == HODLR_F64)
    s = logdet_grad_impl<float, double>(F, st, M, dD, dU, dV);
  else
    s = logdet_grad_impl<float, float>(F, st, M, dD, dU, dV);
  // the temporaries are released once the stream has used them
  if (hipStreamSynchronize(st) != hipSuccess && s == HODLR_OK) s = HODLR_ERR_HIP;
  M.release();
  return s;
}

size_t hodlr_factor_bytes(const hodlr_factors* Fc) {
  if (!Fc) return 0;
  hodlr_factors* F = const_cast<hodlr_factors*>(Fc);
  std::lock_guard<std::mutex> g(F->mu);
  size_t b = F->mem.bytes + F->emb.bytes;
  for (auto& kv : F->wsmap) b += kv.second->mem.bytes;
  return b;
}

void hodlr_destroy(hodlr_factors* F) {
  if (!F) return;
  // wait only for this factorization's own work: the factorization itself and
  // the last call on each stream that used it
  hipEventSynchronize(F->ready);
  hipEventSynchronize(F->na_done);
  for (auto& kv : F->wsmap) {
    hipEventSynchronize(kv.second->done);
    kv.second->mem.release();
    hipEventDestroy(kv.second->done);
  }
  F->wsmap.clear();
  F->mem.release();
  F->emb.release();
  hipEventDestroy(F->ready);
  hipEventDestroy(F->na_done);
  delete F;
}

const char* hodlr_status_string(hodlr_status s) {
  switch (s) {
    case HODLR_OK: return "ok";
    case HODLR_ERR_ARG: return "invalid argument";
    case HODLR_ERR_ALLOC: return "device allocation failed";
    case HODLR_ERR_HIP: return "HIP runtime error";
    case HODLR_ERR_UNSUPPORTED: return "unsupported by this build";
    case HODLR_ERR_SINGULAR: return "exactly singular pivot";
    case HODLR_ERR_NOT_CONVERGED: return "iterative refinement did not converge";
  }
  return "unknown status";
}

void hodlr_timing_enable(int32_t enable) {
  std::lock_guard<std::mutex> g(g_tmu);
  if (enable) {
    drain_records();
    g_tot.clear();
  }
  g_timing = enable != 0;
}

int32_t hodlr_kernel_times(const char** names, double* total_ms, int64_t* launches, int32_t cap) {
  std::lock_guard<std::mutex> g(g_tmu);
  drain_records();
  int32_t i = 0;
  for (auto& kv : g_tot) {
    if (i < cap) {
      if (names) names[i] = kv.first.c_str();
      if (total_ms) total_ms[i] = kv.second.first;
      if (launches) launches[i] = kv.second.second;
    }
    ++i;
  }
  return i;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// construction by cross approximation
// ---------------------------------------------------------------------------
extern "C" {

hodlr_status hodlr_construct(const hodlr_kernel* k, int64_t n, int32_t levels, const int64_t* leaf_offsets,
                             const int32_t* ranks, hodlr_dtype dtype, void* D, int64_t ldd, void* U, int64_t ldu,
                             void* V, int64_t ldv, void* stream) {
  if (!k || !k->points) return HODLR_ERR_ARG;
  if (k->kind == HODLR_KERNEL_LAPLACE_DL) {
    if (k->dim != 2 || !k->normals || !k->weights || !k->curvature) return HODLR_ERR_ARG;
  } else if (k->kind == HODLR_KERNEL_GAUSS || k->kind == HODLR_KERNEL_MATERN32) {
    if (k->dim < 1 || k->dim > 3 || !(k->ell > 0.0) || !std::isfinite(k->ell)) return HODLR_ERR_ARG;
  } else {
    return HODLR_ERR_ARG;
  }
  if (k->ldp < n || !std::isfinite(k->shift)) return HODLR_ERR_ARG;
  if (n >= (int64_t(1) << 31)) return HODLR_ERR_UNSUPPORTED;
  hodlr_matrix A{n, levels, leaf_offsets, ranks, dtype, D, ldd, U, ldu, V, ldv};
  std::vector<int64_t> off;
  std::vector<int> rk;
  int m_max = 0;
  hodlr_status s = validate(&A, off, rk, m_max);
  if (s) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int L = levels;
  int R = 0, kmax = 0;
  for (int r : rk) {
    R += r;
    kmax = std::max(kmax, r);
  }
  hodlr::ConstructKernel kd{(int)k->kind, k->dim, k->points, k->ldp, k->normals, k->weights, k->curvature, k->ell,
                            k->shift};
  DevMem M;
  auto run = [&]() -> hodlr_status {
    hodlr_status e;
    int64_t* d_off = nullptr;
    if ((e = M.alloc(&d_off, off.size()))) return e;
    if (hipMemcpyAsync(d_off, off.data(), off.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess)
      return HODLR_ERR_HIP;
    const int nleaf = 1 << L;
    if (dtype == HODLR_F64)
      HL("construct_leaves",
         hodlr::launch_construct_leaves<double>(st, kd, nleaf, d_off, m_max, static_cast<double*>(D), ldd));
    else
      HL("construct_leaves",
         hodlr::launch_construct_leaves<float>(st, kd, nleaf, d_off, m_max, static_cast<float*>(D), ldd));
    if (R == 0) return HODLR_OK;
    // the sibling blocks of every level and their tiles
    const int te = hodlr::aca_tile_elems();
    std::vector<hodlr::AcaBlock> blocks;
    std::vector<hodlr::AcaTile> tiles;
    int col = 0;
    for (int l = 1; l <= L; ++l) {
      const int r = rk[l - 1];
      if (r > 0) {
        const int per = 1 << (L - l);
        for (int a = 0; a < (1 << l); ++a) {
          const int b = a ^ 1;
          hodlr::AcaBlock B;
          B.r0 = off[(size_t)a * per];
          B.m = (int32_t)(off[(size_t)(a + 1) * per] - B.r0);
          B.c0 = off[(size_t)b * per];
          B.n = (int32_t)(off[(size_t)(b + 1) * per] - B.c0);
          B.col = col;
          B.rank = r;
          B.tile0 = (int32_t)tiles.size();
          B.ntile = (std::max(B.m, B.n) + te - 1) / te;
          for (int t = 0; t < B.ntile; ++t) tiles.push_back({(int32_t)blocks.size(), t, (int32_t)tiles.size()});
          blocks.push_back(B);
        }
      }
      col += r;
    }
    const size_t nt = tiles.size();
    hodlr::AcaBlock* d_blocks = nullptr;
    hodlr::AcaTile* d_tiles = nullptr;
    hodlr::AcaPartials P{};
    if ((e = M.alloc(&d_blocks, blocks.size())) || (e = M.alloc(&d_tiles, nt)) || (e = M.alloc(&P.rp_abs, nt)) ||
        (e = M.alloc(&P.rp_val, nt)) || (e = M.alloc(&P.rp_idx, nt)) || (e = M.alloc(&P.cp_abs, nt)) ||
        (e = M.alloc(&P.cp_idx, nt)) || (e = M.alloc(&P.piv, blocks.size() * kmax)))
      return e;
    if (hipMemcpyAsync(d_blocks, blocks.data(), blocks.size() * sizeof(hodlr::AcaBlock), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(d_tiles, tiles.data(), nt * sizeof(hodlr::AcaTile), hipMemcpyHostToDevice, st) != hipSuccess)
      return HODLR_ERR_HIP;
    double* U64 = static_cast<double*>(U);
    double* V64 = static_cast<double*>(V);
    int64_t ldu64 = ldu, ldv64 = ldv;
    if (dtype == HODLR_F32) {
      if ((e = M.alloc(&U64, (size_t)n * R)) || (e = M.alloc(&V64, (size_t)n * R))) return e;
      ldu64 = ldv64 = n;
    }
    for (int step = 0; step < kmax; ++step)
      HL("aca_step", hodlr::launch_aca_step(st, kd, (int)nt, d_blocks, d_tiles, step, kmax, U64, ldu64, V64, ldv64, P));
    if (dtype == HODLR_F32) {
      HL("construct_store", hodlr::launch_store_cols<float>(st, n, R, U64, ldu64, static_cast<float*>(U), ldu));
      HL("construct_store", hodlr::launch_store_cols<float>(st, n, R, V64, ldv64, static_cast<float*>(V), ldv));
    }
    return HODLR_OK;
  };
  s = run();
  // the host vectors the copies read and the temporaries live until the stream is done
  if (hipStreamSynchronize(st) != hipSuccess && s == HODLR_OK) s = HODLR_ERR_HIP;
  M.release();
  return s;
}

}  // extern "C"
