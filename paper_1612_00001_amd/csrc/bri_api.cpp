// C ABI (include/bri.h) and the plan executor.
//
// A plan (bri_plan.cpp) is a list of batched steps over b x b workspace
// slots.  The executor resolves every operand to a device view, writes all
// work descriptors of one call into a pinned host buffer, uploads them with a
// single copy into the caller's workspace and then enqueues the kernels of
// every step on the caller's stream.  Nothing is allocated on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <tuple>

#include "../../include/bri.h"
#include "bri_internal.h"
#include "bri_kernels.h"
#include "bri_refine.h"

namespace bri {
namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  std::vector<int> nfast;        // explicit GEMM steps: items taking the fast kernel instance
  std::vector<int> ndirect;      // of those, the leading items that qualify for the direct-to-LDS instance
  size_t slot_bytes = 0;
  size_t slots_off = 0, perm_off = 0, swap_off = 0, aux_off = 0, aux_bytes = 0, info_off = 0, desc_off = 0;
  size_t desc_bytes = 0;
  size_t total = 0;
  std::vector<size_t> step_off;  // descriptor offset of every step (relative to desc_off)
};

size_t item_bytes(StepKind k) {
  switch (k) {
    case ST_LOAD:
      return sizeof(LoadItem);
    case ST_GETRF:
    case ST_TRTRI:
      return sizeof(LuItem);
    default:
      return sizeof(GemmItem);
  }
}

Layout make_layout(const Plan& p, int elem) {
  Layout L;
  const size_t b = static_cast<size_t>(p.b);
  L.slot_bytes = align_up(b * b * elem);
  size_t off = 0;
  L.slots_off = off;
  off += L.slot_bytes * p.nslots;
  L.perm_off = off;
  off += align_up(b * sizeof(int32_t) * p.nslots);
  L.swap_off = off;
  off += align_up(sizeof(int32_t) * kSwapWords * p.nslots);
  L.aux_off = off;
  L.aux_bytes = align_up(static_cast<size_t>(kAuxElems) * elem);
  off += L.aux_bytes * p.nslots;
  L.info_off = off;
  off += kAlign;
  L.desc_off = off;
  size_t d = 0;
  for (const Step& s : p.steps) {
    L.step_off.push_back(d);
    d += align_up(item_bytes(s.kind) * s.items.size());
  }
  L.desc_bytes = d;
  off += d;
  L.total = off;
  return L;
}

struct CachedPlan {
  Plan plan;
  Layout layout;
  void* host = nullptr;  // pinned descriptor staging buffer
  hipEvent_t uploaded = nullptr;
  std::mutex mu;
  // The last call's work captured as a HIP graph (upload, status clear and
  // every kernel), replayed while a call's descriptors and launch settings
  // are byte for byte those of the captured one.
  hipGraphExec_t graph = nullptr;
  std::vector<char> graph_desc;  // descriptors (and settings) the graph was captured with
  ~CachedPlan() {
    if (graph) (void)hipGraphExecDestroy(graph);
    if (uploaded) (void)hipEventDestroy(uploaded);
    if (host) (void)hipHostFree(host);
  }
};

typedef std::tuple<int, int64_t, int, int, int, int, int, int> PlanKey;  // kind,n,k,i,j,width,elem,transpose
// kind: 0 block plan, 1 block column plan, 2 block plan with kept pivots,
// 3 block plan reading M through staged block loads only, 4 block plan in
// the literal frame order

std::mutex g_cache_mu;
std::map<PlanKey, std::shared_ptr<CachedPlan>>& cache() {
  static std::map<PlanKey, std::shared_ptr<CachedPlan>> c;
  return c;
}

int elem_size(int precision) { return precision == BRI_F32 ? 4 : 8; }
// Element size of the workspace slots: the mixed paths keep their recursion in float.
int slot_elem_size(int precision) { return precision == BRI_F64 ? 8 : 4; }

int64_t leaves_of(int k) { return static_cast<int64_t>(std::pow(4.0, std::max(0, k - 2))); }

int auto_width(int64_t n, int k, int precision) {
  const int64_t b = (n + k - 1) / k;
  const int64_t tiles = ((b + 127) / 128) * ((b + 127) / 128);
  // At least enough independent Schur operations for ~2048 output tiles of
  // 128 x 128, rounded up to a power of 4 (the lock-step batch sizes); deeper
  // recursions (more leaves) go wider, up to 256 nodes side by side, because
  // every lock-step batch pays one factorisation latency.
  int64_t w = 1;
  while (w * tiles < 2048) w *= 4;
  while (w < 256 && w * 4 <= leaves_of(k) && w * 16 <= leaves_of(k)) w *= 4;
  // Keep the live workspace within 48 GiB, a sixth of the MI355X's 288 GB
  // of HBM: about (k + 4) / 2 blocks per branch evaluated side by side
  // (measured: 6.0 at k = 8, W = 64; 5.0 at W = 256).  At n = 16384, k = 8 in
  // FP64 this allows W = 256 (40 GiB): a quarter as many lock-step batches,
  // and so factorisation latencies, as W = 64 (4.84 s -> 4.65 s per call).
  const double per = 0.5 * (k + 4) * b * b * slot_elem_size(precision);
  int64_t wmem = 1;
  while (wmem * 4 * per <= 48.0 * (1ull << 30)) wmem *= 4;
  w = std::min(w, wmem);
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(w, leaves_of(k))));
}

// Plan kind of a single-block call (see get_plan); the literal frame order
// exists for the plain precisions without kept pivots only (order_ok).
int block_kind(const bri_opts* o) { return o->order == BRI_ORDER_PAPER ? 4 : (o->reuse ? 2 : 0); }
bool order_ok(const bri_opts* o) {
  if (o->order == BRI_ORDER_PRINCIPAL) return true;
  return o->order == BRI_ORDER_PAPER && !o->reuse && (o->precision == BRI_F64 || o->precision == BRI_F32);
}

int resolve_width(int64_t n, int k, const bri_opts* o) {
  if (o && o->concurrency > 0) return static_cast<int>(std::min<int64_t>(o->concurrency, leaves_of(k)));
  return auto_width(n, k, o ? o->precision : BRI_F64);
}

// With a workspace budget and automatic concurrency, a copy of *o whose
// concurrency is the widest width (the automatic one, then down by factors
// of 4) whose workspace, as size() computes it for the copy, fits the
// budget; fits = false when even width 1 does not.
template <typename F>
bri_opts with_budget(const bri_opts* o, int64_t n, int k, F size, bool& fits) {
  bri_opts r = *o;
  fits = true;
  if (o->workspace_budget == 0 || o->concurrency > 0) return r;
  int w = auto_width(n, k, o->precision);
  for (;;) {
    r.concurrency = w;
    size_t s = 0;
    try {
      s = size(r);
    } catch (const std::exception&) {
      s = 0;
    }
    if (s != 0 && s <= o->workspace_budget) return r;
    if (w <= 1) {
      fits = false;
      return r;
    }
    w = std::max(1, w / 4);
  }
}

std::shared_ptr<CachedPlan> get_plan(int kind, int64_t n, int k, int i, int j, int width, int elem, int transpose) {
  PlanKey key(kind, n, k, i, j, width, elem, transpose);
  std::lock_guard<std::mutex> g(g_cache_mu);
  auto& c = cache();
  auto itp = c.find(key);
  if (itp != c.end()) return itp->second;
  auto cp = std::make_shared<CachedPlan>();
  cp->plan = kind == 0   ? make_block_plan(n, k, i, j, width)
             : kind == 2 ? make_block_plan_reuse(n, k, i, j, width)
             : kind == 3 ? make_block_plan_staged(n, k, i, j, width)
             : kind == 4 ? make_block_plan_literal(n, k, i, j, width)
                         : make_column_plan(n, k, j, width);
  cp->plan.transpose = transpose;
  cp->layout = make_layout(cp->plan, elem);
  if (c.size() > 64) c.clear();
  c[key] = cp;
  return cp;
}

// ---------------------------------------------------------------------------
// Operand resolution
// ---------------------------------------------------------------------------
struct Ctx {
  int pivoting = BRI_PIVOT_TILE;
  int lu = 0;           // factorisation variant (bri_opts::factorization)
  const char* M = nullptr;
  int64_t n = 0, ldm = 0;
  int b = 0;
  int elem = 8;
  int transpose = 0;
  char* ws = nullptr;
  const Layout* lay = nullptr;
  char* out = nullptr;
  int64_t ldo = 0;
  int32_t* info = nullptr;
  char* rhs = nullptr;  // right-hand side of a solve plan (OPND_RHS), (k b) x b
  int64_t ldr = 0;
  int lp = 0;           // float products: 0 FP32 MFMA, 1 FP16 split, 2 BF16 split
  bool wide = false;    // float recursion whose tile factorisations compute in double
  int m_elem = 0;       // element size of M when it differs from elem (mixed: double M, float plan)
  const double* m_max = nullptr;  // mixed: max |M| on the device (blocks of M read scaled)
  const RbfSource* rbf = nullptr;  // matrix-free M: its description on the device
  unsigned long long* stats = nullptr;  // device accounting (bri_opts::d_stats), or null
  const char* stats_base = nullptr;     // the caller's workspace and its size
  uint64_t stats_limit = 0;
};

// How the kernels of a plan are launched.
struct ExecCfg {
  int pivoting = BRI_PIVOT_TILE;
  int lu = 0;           // factorisation variant (bri_opts::factorization)
  int lp = 0;           // float products: 0 FP32 MFMA, 1 FP16 split, 2 BF16 split
  bool wide = false;    // tile factorisations of float matrices in double
  int32_t* range_flag = nullptr;  // FP16 split products: operand outside the FP16 range
  char* split = nullptr;          // split FP16 / BF16 products: scratch for operands split once
  size_t split_bytes = 0;
  unsigned long long* stats = nullptr;  // device accounting of the executed steps, or null
  const char* stats_base = nullptr;
  uint64_t stats_limit = 0;
};
ExecCfg cfg_of(const Ctx& c) {
  return ExecCfg{c.pivoting, c.lu, c.lp, c.wide, nullptr, nullptr, 0, c.stats, c.stats_base, c.stats_limit};
}

DView zero_view() {
  DView v;
  v.p = nullptr;
  v.ld = 0;
  v.rowperm = nullptr;
  v.rows = 0;
  v.cols = 0;
  v.diag = INT_MIN / 2;
  v.trans = 0;
  v.tri = 0;
  v.src64_max = nullptr;
  v.rbf = nullptr;
  v.r0 = v.c0 = 0;
  return v;
}

char* slot_ptr(const Ctx& c, int s) { return c.ws + c.lay->slots_off + c.lay->slot_bytes * s; }
int32_t* perm_ptr(const Ctx& c, int s) {
  return reinterpret_cast<int32_t*>(c.ws + c.lay->perm_off) + static_cast<int64_t>(s) * c.b;
}
int32_t* swap_ptr(const Ctx& c, int s) {
  return reinterpret_cast<int32_t*>(c.ws + c.lay->swap_off) + static_cast<int64_t>(s) * kSwapWords;
}
char* aux_ptr(const Ctx& c, int s) { return c.ws + c.lay->aux_off + c.lay->aux_bytes * s; }

DView slot_view(const Ctx& c, int s, int tri = 0) {
  DView v = zero_view();
  v.p = slot_ptr(c, s);
  v.ld = c.b;
  v.rows = c.b;
  v.cols = c.b;
  v.tri = static_cast<int16_t>(tri);
  return v;
}

DView resolve(const Ctx& c, const Opnd& o) {
  DView v = zero_view();
  const int64_t b = c.b;
  switch (o.kind) {
    case OPND_SLOT:
      return slot_view(c, o.a);
    case OPND_MBLK: {
      const int64_t r = o.a, col = o.b;
      const int64_t rows = std::max<int64_t>(0, std::min<int64_t>(b, c.n - r * b));
      const int64_t cols = std::max<int64_t>(0, std::min<int64_t>(b, c.n - col * b));
      v.rows = static_cast<int32_t>(rows);
      v.cols = static_cast<int32_t>(cols);
      v.diag = static_cast<int32_t>(col * b - r * b);
      v.ld = c.ldm;
      if (rows > 0 && cols > 0) {
        // Block (r, c) of Gamma, or of Gamma^T (stored transposed).
        const int64_t off = c.transpose ? (col * b) * c.ldm + r * b : (r * b) * c.ldm + col * b;
        v.p = c.M + off * (c.m_elem ? c.m_elem : c.elem);
      } else {
        v.p = c.M;
      }
      v.trans = static_cast<int16_t>(c.transpose ? 1 : 0);
      v.src64_max = c.m_max;
      if (c.rbf) {
        v.rbf = c.rbf;
        v.p = c.rbf;  // not read: the elements are evaluated
        v.r0 = static_cast<int32_t>(r * b);
        v.c0 = static_cast<int32_t>(col * b);
      }
      return v;
    }
    case OPND_IDENT:
      v.diag = 0;
      return v;
    case OPND_OUT:
      v.p = c.out + static_cast<int64_t>(o.a) * b * c.ldo * c.elem;
      v.ld = c.ldo;
      v.rows = c.b;
      v.cols = c.b;
      return v;
    case OPND_RHS:
      if (!c.rhs) throw std::logic_error("solve plan without a right-hand side");
      v.p = c.rhs + static_cast<int64_t>(o.a) * b * c.ldr * c.elem;
      v.ld = c.ldr;
      v.rows = c.b;
      v.cols = c.b;
      return v;
    default:
      return v;
  }
}

void* dst_ptr(const Ctx& c, const Opnd& o, int64_t& ld) {
  if (o.kind == OPND_SLOT) {
    ld = c.b;
    return slot_ptr(c, o.a);
  }
  if (o.kind == OPND_OUT) {
    ld = c.ldo;
    return c.out + static_cast<int64_t>(o.a) * c.b * c.ldo * c.elem;
  }
  throw std::logic_error("bad destination operand");
}

GemmItem gemm_base(const Ctx& c) {
  GemmItem g;
  std::memset(&g, 0, sizeof(g));
  g.A = g.B = g.Cin = g.Sub = zero_view();
  g.M = g.N = g.K = c.b;
  return g;
}

// Work descriptors of one plan step for context c, appended to the vectors
// (product items split into those the direct-to-LDS instance can take, the
// other ones the fast instance takes, and the rest).
struct StepItems {
  std::vector<LoadItem> loads;
  std::vector<LuItem> lus;
  std::vector<GemmItem> direct, fast, slow;
  void clear() {
    loads.clear();
    lus.clear();
    direct.clear();
    fast.clear();
    slow.clear();
  }
  size_t count() const { return loads.size() + lus.size() + direct.size() + fast.size() + slow.size(); }
  int nfast() const { return static_cast<int>(direct.size() + fast.size()); }
  int ndirect() const { return static_cast<int>(direct.size()); }
  // Writes the items to dst (direct, then fast products first); returns the
  // bytes written.
  size_t write(char* dst) const {
    size_t off = 0;
    auto put = [&](const void* src, size_t bytes) {
      std::memcpy(dst + off, src, bytes);
      off += bytes;
    };
    put(loads.data(), loads.size() * sizeof(LoadItem));
    put(lus.data(), lus.size() * sizeof(LuItem));
    put(direct.data(), direct.size() * sizeof(GemmItem));
    put(fast.data(), fast.size() * sizeof(GemmItem));
    put(slow.data(), slow.size() * sizeof(GemmItem));
    return off;
  }
};

void describe_step(const Ctx& c, const Step& s, StepItems& out) {
  for (const StepItem& it : s.items) {
    switch (s.kind) {
      case ST_LOAD: {
        LoadItem li;
        std::memset(&li, 0, sizeof(li));
        li.src = resolve(c, it.x);
        li.dst = dst_ptr(c, it.dst, li.ldd);
        li.rows = c.b;
        li.cols = c.b;
        out.loads.push_back(li);
        break;
      }
      case ST_GETRF:
      case ST_TRTRI: {
        LuItem lu;
        std::memset(&lu, 0, sizeof(lu));
        lu.a = slot_ptr(c, it.dst.a);
        lu.perm = perm_ptr(c, it.dst.a);
        lu.swaps = swap_ptr(c, it.dst.a);
        // scratch of the triangular inversion, or the shadow of the recursive LU
        lu.tmp = it.x.kind == OPND_SLOT ? slot_ptr(c, it.x.a) : nullptr;
        lu.aux = aux_ptr(c, it.dst.a);
        lu.info = c.info;
        lu.node = it.node;
        lu.b = c.b;
        out.lus.push_back(lu);
        break;
      }
      default: {
        // A matrix in another precision is read through load steps only.
        if ((c.m_max || c.rbf) && (it.x.kind == OPND_MBLK || it.y.kind == OPND_MBLK || it.cin.kind == OPND_MBLK ||
                                   it.sub.kind == OPND_MBLK))
          throw std::logic_error("unstaged block of M in a product");
        GemmItem g = gemm_base(c);
        g.out = dst_ptr(c, it.dst, g.ldo);
        if (s.kind == ST_TRMM_L) {
          g.A = slot_view(c, it.x.a, 1);
          g.B = resolve(c, it.y);
          g.B.rowperm = perm_ptr(c, it.x.a);
          g.alpha = 1.0;
        } else if (s.kind == ST_TRMM_U) {
          g.A = slot_view(c, it.x.a, 2);
          g.B = resolve(c, it.y);
          g.alpha = 1.0;
        } else {
          g.A = resolve(c, it.x);
          g.B = resolve(c, it.y);
          if (it.cin.kind != OPND_NONE) {
            g.Cin = resolve(c, it.cin);
            g.has_cin = 1;
            g.beta = 1.0;
          }
          if (it.sub.kind != OPND_NONE) {
            g.Sub = resolve(c, it.sub);
            g.has_sub = 1;
          }
          g.alpha = (s.kind == ST_GEMM_ACC) ? 1.0 : -1.0;
        }
        // direct: the FP64 direct-to-LDS instance, or for the split FP16 /
        // BF16 products of float storage the vectorised and split-once ones
        const bool direct = c.elem == 8 ? gemm_item_is_direct(g, 8) : (c.lp >= 1 && gemm_item_is_lp_vec(g));
        if (!gemm_item_is_fast(g))
          out.slow.push_back(g);
        else
          (direct ? out.direct : out.fast).push_back(g);
        break;
      }
    }
  }
}

void build_descriptors(const Ctx& c, const Plan& p, char* host, std::vector<int>& nfast, std::vector<int>& ndirect) {
  nfast.assign(p.steps.size(), 0);
  ndirect.assign(p.steps.size(), 0);
  StepItems items;
  for (size_t si = 0; si < p.steps.size(); ++si) {
    items.clear();
    describe_step(c, p.steps[si], items);
    items.write(host + c.lay->step_off[si]);
    nfast[si] = items.nfast();
    ndirect[si] = items.ndirect();
  }
}

// ---------------------------------------------------------------------------
// Step timing (bri_profile_*)
// ---------------------------------------------------------------------------
struct ProfRecord {
  int kind;
  int64_t launches;
  double flops;
  hipEvent_t e0, e1;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRecord> g_prof_pending;
std::vector<hipEvent_t> g_prof_pool;
bri_profile_entry g_prof_acc[BRI_PROFILE_KINDS];

hipEvent_t prof_event() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

double step_flops(const Step& s, int b) {
  const double b3 = static_cast<double>(b) * b * b;
  const double n = static_cast<double>(s.items.size());
  switch (s.kind) {
    case ST_LOAD:
      return 0.0;
    case ST_GETRF:
      return n * getrf_flops(b);
    case ST_TRTRI:
      return n * trtri_flops(b);
    case ST_TRMM_L:
    case ST_TRMM_U:
      return n * b3;
    default:
      return n * 2.0 * b3;
  }
}

int64_t step_launches(StepKind kind, int count, int b, int pivoting, bool uniform, int lu) {
  switch (kind) {
    case ST_GETRF:
      return getrf_launches(b, lu_kind(count, b, pivoting == BRI_PIVOT_PANEL, uniform, lu));
    case ST_TRTRI:
      return trtri_launches(b, lu_kind(count, b, pivoting == BRI_PIVOT_PANEL, uniform, lu));
    default:
      return 1;
  }
}

// One step as launched: its kind, item count, fast product items, descriptor
// address on the device and the step it stands for (for the profile record).
struct ExecStep {
  StepKind kind;
  int count;
  int nfast;
  int ndirect;
  const void* desc;
  const Step* step;
  double flops;  // algorithmic flops of all items (profile record)
  bool uniform;  // every item has the block order bmax
};

// The LU variant of a step's factorisation (lu_kind); the triangular
// inversion after it runs only after the tile-step and panel LUs (the
// recursive LU leaves the factors inverted).
LuKind step_lu(const ExecStep& s, int bmax, int pivoting, int lu) {
  return lu_kind(s.count, bmax, pivoting == BRI_PIVOT_PANEL, s.uniform, lu);
}
bool step_inverts_factors(const ExecStep& s, int bmax, int pivoting, int lu) {
  return step_lu(s, bmax, pivoting, lu) == LU_RECURSIVE;
}

// Enqueues the kernels of the steps; bmax is the largest block order among
// the items (merged batches mix orders; every kernel skips the parts of a
// smaller matrix).
template <typename T>
int run_exec(const std::vector<ExecStep>& steps, int bmax, const ExecCfg& cfg, hipStream_t st) {
  const int pivoting = cfg.pivoting, lu = cfg.lu, lp = cfg.lp;
  bool prof;
  {
    std::lock_guard<std::mutex> g(g_prof_mu);
    prof = g_prof_on;
  }
  for (const ExecStep& s : steps) {
    if (s.count <= 0) continue;
    hipError_t e = hipSuccess;
    ProfRecord rec{};
    if (prof) {
      std::lock_guard<std::mutex> g(g_prof_mu);
      rec.kind = s.kind;
      rec.launches = step_launches(s.kind, s.count, bmax, pivoting, s.uniform, lu);
      // a triangular inversion skipped after the recursive LU counts no work
      rec.flops = s.kind == ST_TRTRI && step_inverts_factors(s, bmax, pivoting, lu) ? 0.0 : s.flops;
      rec.e0 = prof_event();
      rec.e1 = prof_event();
      if (!rec.e0 || !rec.e1 || hipEventRecord(rec.e0, st) != hipSuccess) return BRI_ERR_HIP;
    }
    switch (s.kind) {
      case ST_LOAD:
        e = launch_load<T>(static_cast<const LoadItem*>(s.desc), s.count, bmax, bmax, st);
        break;
      case ST_GETRF: {
        const LuItem* d = static_cast<const LuItem*>(s.desc);
        switch (step_lu(s, bmax, pivoting, lu)) {
          case LU_PANEL: e = launch_getrf<T>(d, s.count, bmax, st); break;
          case LU_RECURSIVE: e = launch_getrf_rec<T>(d, s.count, bmax, cfg.wide, lp, cfg.range_flag, st); break;
          default: e = launch_getrf_tile<T>(d, s.count, bmax, cfg.wide, st); break;
        }
        break;
      }
      case ST_TRTRI:
        // after the recursive LU the factors are already inverted
        if (!step_inverts_factors(s, bmax, pivoting, lu))
          e = launch_trtri<T>(static_cast<const LuItem*>(s.desc), s.count, bmax, pivoting != BRI_PIVOT_PANEL, st);
        break;
      default: {
        GemmLaunch L{};
        L.mode = GEMM_EXPLICIT;
        L.elem = sizeof(T);
        L.items = s.desc;
        L.count = s.count;
        L.w = s.nfast;
        L.ndl = s.ndirect;
        L.lp = lp;
        L.tri = (s.kind == ST_TRMM_L || s.kind == ST_TRMM_U) ? 1 : 0;
        L.range_flag = cfg.range_flag;
        L.split = cfg.split;
        L.split_bytes = static_cast<int64_t>(cfg.split_bytes);
        e = launch_gemm<T>(L, bmax, bmax, st);
        break;
      }
    }
    if (e != hipSuccess) return BRI_ERR_HIP;
    if (cfg.stats && launch_stats(s.kind, s.desc, s.count, sizeof(T), cfg.stats, cfg.stats_base, cfg.stats_limit,
                                  st) != hipSuccess)
      return BRI_ERR_HIP;
    if (prof) {
      std::lock_guard<std::mutex> g(g_prof_mu);
      if (hipEventRecord(rec.e1, st) != hipSuccess) return BRI_ERR_HIP;
      g_prof_pending.push_back(rec);
    }
  }
  return BRI_OK;
}

template <typename T>
int run_steps(const Ctx& c, const Plan& p, hipStream_t st) {
  const char* dbase = c.ws + c.lay->desc_off;
  std::vector<ExecStep> ex;
  ex.reserve(p.steps.size());
  for (size_t si = 0; si < p.steps.size(); ++si) {
    const Step& s = p.steps[si];
    ex.push_back(ExecStep{s.kind, static_cast<int>(s.items.size()), c.lay->nfast[si], c.lay->ndirect[si],
                          dbase + c.lay->step_off[si], &s,
                          step_flops(s, c.b), true});
  }
  return run_exec<T>(ex, c.b, cfg_of(c), st);
}

// Descriptor staging of the calls that allocate nothing (invert_block_noalloc):
// one static, pageable host buffer.  hipMemcpyAsync returns once a pageable
// source has been taken (staged for the transfer), so the next call may
// overwrite it; the mutex keeps host threads apart.
constexpr size_t kNoallocDescBytes = size_t(8) << 20;
alignas(64) char g_noalloc_desc[kNoallocDescBytes];
std::mutex g_noalloc_mu;

// Enqueues the status clear, the descriptor upload (from cp.host) and the
// kernels of plan cp on st.
int enqueue_call(CachedPlan& cp, Ctx& c, bool clear_info, hipStream_t st) {
  if (clear_info && launch_fill_int(c.info, 1, 0, st) != hipSuccess) return BRI_ERR_HIP;
  if (c.stats && launch_fill_int(reinterpret_cast<int32_t*>(c.stats), 8, 0, st) != hipSuccess) return BRI_ERR_HIP;
  if (cp.layout.desc_bytes > 0) {
    if (hipMemcpyAsync(c.ws + cp.layout.desc_off, cp.host, cp.layout.desc_bytes, hipMemcpyHostToDevice, st) !=
        hipSuccess)
      return BRI_ERR_HIP;
  }
  if (hipEventRecord(cp.uploaded, st) != hipSuccess) return BRI_ERR_HIP;
  return c.elem == 8 ? run_steps<double>(c, cp.plan, st) : run_steps<float>(c, cp.plan, st);
}

// Graph capture of whole calls: for plans with few launches (where the
// launch overhead counts), never while step timing is on.
constexpr int64_t kGraphMaxLaunches = 4096;
bool graph_eligible(const CachedPlan& cp) {
  {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (g_prof_on) return false;
  }
  return cp.plan.launches <= kGraphMaxLaunches && cp.layout.desc_bytes > 0;
}

// Everything a captured call depends on: its descriptors (which hold every
// operand, output and status address) and the launch settings.
std::vector<char> graph_key(const CachedPlan& cp, const Ctx& c, bool clear_info) {
  std::vector<char> key(static_cast<const char*>(cp.host), static_cast<const char*>(cp.host) + cp.layout.desc_bytes);
  struct Settings {
    const void* ws;
    const void* info;
    int pivoting, lu, lp, elem, b, clear;
  } st_{c.ws, c.info, c.pivoting, c.lu, c.lp, c.elem, c.b, clear_info ? 1 : 0};
  const char* p = reinterpret_cast<const char*>(&st_);
  key.insert(key.end(), p, p + sizeof(st_));
  for (size_t s = 0; s < cp.layout.nfast.size(); ++s) {
    const int32_t v[2] = {cp.layout.nfast[s], cp.layout.ndirect[s]};
    key.insert(key.end(), reinterpret_cast<const char*>(v), reinterpret_cast<const char*>(v) + sizeof(v));
  }
  return key;
}

// A library-owned stream of the current device to capture on (the caller's
// stream may be the legacy default stream, which cannot be captured).
hipStream_t capture_stream() {
  static std::mutex mu;
  static hipStream_t per_device[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  if (!per_device[dev] && hipStreamCreateWithFlags(&per_device[dev], hipStreamNonBlocking) != hipSuccess)
    per_device[dev] = nullptr;
  return per_device[dev];
}

// One capture at a time on the library's capture stream.
std::mutex g_capture_mu;

// The call's work captured into an executable graph (not run), or null.
hipGraphExec_t capture_call(CachedPlan& cp, Ctx& c, bool clear_info) {
  hipStream_t cs = capture_stream();
  if (!cs) return nullptr;
  std::lock_guard<std::mutex> cap(g_capture_mu);
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
  bool ok = true;
  if (clear_info) ok = launch_fill_int(c.info, 1, 0, cs) == hipSuccess;
  if (ok && cp.layout.desc_bytes > 0)
    ok = hipMemcpyAsync(c.ws + cp.layout.desc_off, cp.host, cp.layout.desc_bytes, hipMemcpyHostToDevice, cs) ==
         hipSuccess;
  if (ok) ok = (c.elem == 8 ? run_steps<double>(c, cp.plan, cs) : run_steps<float>(c, cp.plan, cs)) == BRI_OK;
  hipGraph_t graph = nullptr;
  const bool ended = hipStreamEndCapture(cs, &graph) == hipSuccess && graph;
  hipGraphExec_t exec = nullptr;
  if (ok && ended && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) exec = nullptr;
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipGetLastError();  // a failed capture leaves no error behind for later calls
  return ok ? exec : nullptr;
}

// Uploads the descriptors of plan cp for context c and enqueues its kernels.
// noalloc: stage through the static buffer above (no pinned buffer, no event).
int execute(CachedPlan& cp, Ctx& c, hipStream_t st, bool clear_info, bool noalloc = false) {
  c.lay = &cp.layout;
  std::lock_guard<std::mutex> g(cp.mu);
  if (noalloc) {
    if (cp.layout.desc_bytes > kNoallocDescBytes) return BRI_ERR_WORKSPACE;
    std::lock_guard<std::mutex> gn(g_noalloc_mu);
    try {
      build_descriptors(c, cp.plan, g_noalloc_desc, cp.layout.nfast, cp.layout.ndirect);
    } catch (const std::exception&) {
      return BRI_ERR_UNSUPPORTED;
    }
    if (clear_info && launch_fill_int(c.info, 1, 0, st) != hipSuccess) return BRI_ERR_HIP;
    if (c.stats && launch_fill_int(reinterpret_cast<int32_t*>(c.stats), 8, 0, st) != hipSuccess) return BRI_ERR_HIP;
    if (cp.layout.desc_bytes > 0 && hipMemcpyAsync(c.ws + cp.layout.desc_off, g_noalloc_desc, cp.layout.desc_bytes,
                                                   hipMemcpyHostToDevice, st) != hipSuccess)
      return BRI_ERR_HIP;
    return c.elem == 8 ? run_steps<double>(c, cp.plan, st) : run_steps<float>(c, cp.plan, st);
  }
  if (!cp.host) {
    if (hipHostMalloc(&cp.host, std::max<size_t>(cp.layout.desc_bytes, 64)) != hipSuccess) return BRI_ERR_HIP;
    if (hipEventCreateWithFlags(&cp.uploaded, hipEventDisableTiming) != hipSuccess) return BRI_ERR_HIP;
  } else {
    // The previous upload from this staging buffer must have completed.
    if (hipEventSynchronize(cp.uploaded) != hipSuccess) return BRI_ERR_HIP;
  }
  try {
    build_descriptors(c, cp.plan, static_cast<char*>(cp.host), cp.layout.nfast, cp.layout.ndirect);
  } catch (const std::exception&) {
    return BRI_ERR_UNSUPPORTED;
  }
  // The whole call as one graph launch when it repeats the captured one
  // (calls with device accounting launch directly).
  if (graph_eligible(cp) && !c.stats) {
    const std::vector<char> key = graph_key(cp, c, clear_info);
    if (cp.graph && key == cp.graph_desc) {
      if (hipGraphLaunch(cp.graph, st) != hipSuccess) return BRI_ERR_HIP;
      return hipEventRecord(cp.uploaded, st) == hipSuccess ? BRI_OK : BRI_ERR_HIP;
    }
    hipGraphExec_t g = capture_call(cp, c, clear_info);
    if (g) {
      if (cp.graph) (void)hipGraphExecDestroy(cp.graph);
      cp.graph = g;
      cp.graph_desc = key;
      if (hipGraphLaunch(cp.graph, st) != hipSuccess) return BRI_ERR_HIP;
      return hipEventRecord(cp.uploaded, st) == hipSuccess ? BRI_OK : BRI_ERR_HIP;
    }
    // capture failed: run the call directly
  }
  return enqueue_call(cp, c, clear_info, st);
}

bool plain_precision(int p) { return p == BRI_F64 || p == BRI_F32; }
bool mixed_precision(int p) { return p == BRI_MIXED_F32 || p == BRI_MIXED_F16 || p == BRI_MIXED_BF16; }
// Products of the float recursion: FP32 MFMA, or split FP16 / BF16 MFMA.
int lp_of(int p) { return p == BRI_MIXED_F16 ? 1 : (p == BRI_MIXED_BF16 ? 2 : 0); }

// ---------------------------------------------------------------------------
// Pinned staging buffer for the descriptors of batched and mixed calls
// (grown on demand; the event guards reuse while an upload is in flight).
// ---------------------------------------------------------------------------
struct Staging {
  std::mutex mu;
  void* host = nullptr;
  size_t bytes = 0;
  hipEvent_t ev = nullptr;
  // Call with mu held.  Returns nullptr on a HIP failure.
  char* get(size_t need) {
    if (ev && hipEventSynchronize(ev) != hipSuccess) return nullptr;
    if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return nullptr;
    if (bytes < need) {
      if (host) (void)hipHostFree(host);
      host = nullptr;
      bytes = 0;
      if (hipHostMalloc(&host, std::max<size_t>(need, 4096)) != hipSuccess) return nullptr;
      bytes = std::max<size_t>(need, 4096);
    }
    return static_cast<char*>(host);
  }
};
Staging& staging() {
  static Staging s;
  return s;
}

// ---------------------------------------------------------------------------
// Merging plans: members whose plans have the same step structure form a
// group; every step of a group is one launch over the items of all members,
// each item carrying its own block order, operands and status word.
// ---------------------------------------------------------------------------
bool same_structure(const Plan& a, const Plan& b) {
  if (a.steps.size() != b.steps.size()) return false;
  for (size_t s = 0; s < a.steps.size(); ++s)
    if (a.steps[s].kind != b.steps[s].kind || a.steps[s].items.size() != b.steps[s].items.size()) return false;
  return true;
}

struct MergedLayout {
  std::vector<std::vector<int>> groups;       // member indices of every group
  std::vector<std::vector<size_t>> step_off;  // per group and step: descriptor offset
  size_t bytes = 0;
};

MergedLayout merge_layout(const std::vector<const Plan*>& plans) {
  MergedLayout m;
  std::map<size_t, std::vector<int>> by_len;  // step count -> candidate groups
  for (int t = 0; t < static_cast<int>(plans.size()); ++t) {
    std::vector<int>& cands = by_len[plans[t]->steps.size()];
    int g = -1;
    for (int c : cands)
      if (same_structure(*plans[m.groups[c][0]], *plans[t])) g = c;
    if (g < 0) {
      g = static_cast<int>(m.groups.size());
      m.groups.emplace_back();
      cands.push_back(g);
    }
    m.groups[g].push_back(t);
  }
  size_t d = 0;
  for (const std::vector<int>& grp : m.groups) {
    const Plan& p0 = *plans[grp[0]];
    m.step_off.emplace_back();
    for (const Step& st : p0.steps) {
      m.step_off.back().push_back(d);
      d += align_up(item_bytes(st.kind) * st.items.size() * grp.size());
    }
  }
  m.bytes = d;
  return m;
}

// Helper streams of the current device on which the structure groups of a
// merged batch run side by side (created once per device, default priority).
struct GroupStreams {
  static constexpr int kStreams = 4;  // the hardware queues a process gets by default
  std::mutex mu;
  hipStream_t stream[kStreams] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kStreams] = {};
};
GroupStreams* group_streams() {
  static std::mutex mu;
  static GroupStreams* per_device[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  if (!per_device[dev]) {
    auto* gs = new GroupStreams();
    bool ok = hipEventCreateWithFlags(&gs->fork, hipEventDisableTiming) == hipSuccess;
    for (int q = 0; ok && q < GroupStreams::kStreams; ++q)
      ok = hipStreamCreateWithFlags(&gs->stream[q], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&gs->join[q], hipEventDisableTiming) == hipSuccess;
    if (!ok) return nullptr;  // the merged batch then runs on the caller's stream alone
    per_device[dev] = gs;
  }
  return per_device[dev];
}

struct MergedExec {
  std::vector<std::vector<ExecStep>> groups;
  std::vector<int> bmax;
};

// Writes the merged descriptors to host (device copy at dev) and returns the
// steps to launch.  Throws on operands that cannot be resolved.
MergedExec merge_write(const std::vector<const Plan*>& plans, const std::vector<Ctx>& ctx, const MergedLayout& m,
                       char* host, const char* dev) {
  MergedExec ex;
  StepItems items;
  for (size_t g = 0; g < m.groups.size(); ++g) {
    const std::vector<int>& grp = m.groups[g];
    const Plan& p0 = *plans[grp[0]];
    int bmax = 0;
    for (int t : grp) bmax = std::max(bmax, ctx[t].b);
    bool uniform = true;
    for (int t : grp) uniform = uniform && ctx[t].b == bmax;
    ex.bmax.push_back(bmax);
    ex.groups.emplace_back();
    for (size_t si = 0; si < p0.steps.size(); ++si) {
      items.clear();
      double flops = 0;
      for (int t : grp) {
        const Step& st = plans[t]->steps[si];
        describe_step(ctx[t], st, items);
        flops += step_flops(st, ctx[t].b);
      }
      items.write(host + m.step_off[g][si]);
      ex.groups.back().push_back(ExecStep{p0.steps[si].kind, static_cast<int>(items.count()), items.nfast(),
                                          items.ndirect(), dev + m.step_off[g][si], &p0.steps[si], flops, uniform});
    }
  }
  return ex;
}

template <typename T>
int run_merged(const MergedExec& ex, const ExecCfg& cfg, hipStream_t st) {
  bool prof;
  {
    std::lock_guard<std::mutex> g(g_prof_mu);
    prof = g_prof_on;
  }
  GroupStreams* gs = ex.groups.size() > 1 && !prof ? group_streams() : nullptr;
  if (!gs) {
    for (size_t g = 0; g < ex.groups.size(); ++g) {
      const int rc = run_exec<T>(ex.groups[g], ex.bmax[g], cfg, st);
      if (rc != BRI_OK) return rc;
    }
    return BRI_OK;
  }
  // The groups touch disjoint parts of the workspace (each problem its own
  // region and status word, each group its own descriptors, each stream its
  // own share of the split scratch): they run side by side on the helper
  // streams, forked from and joined into st.
  std::lock_guard<std::mutex> lk(gs->mu);
  if (hipEventRecord(gs->fork, st) != hipSuccess) return BRI_ERR_HIP;
  const size_t ns = std::min<size_t>(GroupStreams::kStreams, ex.groups.size());
  for (size_t q = 0; q < ns; ++q)
    if (hipStreamWaitEvent(gs->stream[q], gs->fork, 0) != hipSuccess) return BRI_ERR_HIP;
  const size_t share = cfg.split ? cfg.split_bytes / ns / kAlign * kAlign : 0;
  for (size_t g = 0; g < ex.groups.size(); ++g) {
    ExecCfg gc = cfg;
    gc.split = cfg.split ? cfg.split + share * (g % ns) : nullptr;
    gc.split_bytes = share;
    const int rc = run_exec<T>(ex.groups[g], ex.bmax[g], gc, gs->stream[g % ns]);
    if (rc != BRI_OK) return rc;
  }
  for (size_t q = 0; q < ns; ++q) {
    if (hipEventRecord(gs->join[q], gs->stream[q]) != hipSuccess) return BRI_ERR_HIP;
    if (hipStreamWaitEvent(st, gs->join[q], 0) != hipSuccess) return BRI_ERR_HIP;
  }
  return BRI_OK;
}

// ---------------------------------------------------------------------------
// Plain precisions, batched (tile pivoting): merged block plans.
// ---------------------------------------------------------------------------
int merged_width(int k) { return static_cast<int>(std::min<int64_t>(16, leaves_of(k))); }

struct BatchPlan {
  std::vector<std::shared_ptr<CachedPlan>> plans;  // per problem
  std::vector<size_t> region;                      // per problem: offset of its slot region
  MergedLayout merged;
  size_t info_off = 0, desc_off = 0, total = 0;
};

BatchPlan make_batch_plan(int count, const int64_t* n, const int* k, const int* i, const int* j, int elem,
                          int reuse) {
  BatchPlan bp;
  bp.plans.resize(count);
  bp.region.resize(count);
  std::vector<const Plan*> pl(count);
  size_t off = 0;
  for (int t = 0; t < count; ++t) {
    bp.plans[t] = get_plan(reuse ? 2 : 0, n[t], k[t], i[t], j[t], merged_width(k[t]), elem, 0);
    pl[t] = &bp.plans[t]->plan;
    bp.region[t] = off;
    off += align_up(bp.plans[t]->layout.desc_off);  // slots, permutations, tile scratch, status
  }
  bp.merged = merge_layout(pl);
  bp.info_off = off;  // a status word per problem (when the caller passes no d_info)
  off += align_up(sizeof(int32_t) * count);
  bp.desc_off = off;
  bp.total = off + bp.merged.bytes;
  return bp;
}

template <typename T>
int run_batch(const BatchPlan& bp, const void* const* M, const int64_t* n, const int64_t* ldm, void* const* out,
              const int64_t* ldo, int count, const bri_opts* o) {
  hipStream_t st = o->stream;
  char* ws = static_cast<char*>(o->workspace);
  int32_t* info_words = o->d_info ? o->d_info : reinterpret_cast<int32_t*>(ws + bp.info_off);
  std::vector<Ctx> ctx(count);
  std::vector<const Plan*> pl(count);
  for (int t = 0; t < count; ++t) {
    Ctx& c = ctx[t];
    c.pivoting = BRI_PIVOT_TILE;
    c.M = static_cast<const char*>(M[t]);
    c.n = n[t];
    c.ldm = ldm[t];
    c.b = bp.plans[t]->plan.b;
    c.elem = sizeof(T);
    c.ws = ws + bp.region[t];
    c.lay = &bp.plans[t]->layout;
    c.out = static_cast<char*>(out[t]);
    c.ldo = ldo[t];
    c.info = info_words + t;
    pl[t] = &bp.plans[t]->plan;
  }
  Staging& sg = staging();
  std::lock_guard<std::mutex> lk(sg.mu);
  char* host = sg.get(bp.merged.bytes);
  if (!host) return BRI_ERR_HIP;
  MergedExec ex;
  try {
    ex = merge_write(pl, ctx, bp.merged, host, ws + bp.desc_off);
  } catch (const std::exception&) {
    return BRI_ERR_UNSUPPORTED;
  }
  if (hipMemcpyAsync(ws + bp.desc_off, host, bp.merged.bytes, hipMemcpyHostToDevice, st) != hipSuccess)
    return BRI_ERR_HIP;
  if (hipEventRecord(sg.ev, st) != hipSuccess) return BRI_ERR_HIP;
  if (launch_fill_int(info_words, count, 0, st) != hipSuccess) return BRI_ERR_HIP;
  return run_merged<T>(ex, ExecCfg{BRI_PIVOT_TILE, o->factorization, 0, false, nullptr}, st);
}

// Merged execution of plain precisions needs tile pivoting (the panel
// pivoting kernels assume one block order per launch).
bool batch_mergeable(const bri_opts* o) {
  return (o->pivoting == BRI_PIVOT_TILE || o->pivoting == BRI_PIVOT_AUTO) &&
         (plain_precision(o->precision) || mixed_precision(o->precision));
}

// Status word of a finished call (waits for the stream).
int read_info1(const int32_t* d, int32_t& h, hipStream_t st) {
  h = 0;
  if (hipMemcpyAsync(&h, d, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return BRI_ERR_HIP;
  return BRI_OK;
}

// Status words of a finished call (waits for the stream).
int read_info(const int32_t* d, int count, std::vector<int32_t>& h, hipStream_t st) {
  h.assign(count, 0);
  if (hipMemcpyAsync(h.data(), d, sizeof(int32_t) * count, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return BRI_ERR_HIP;
  return BRI_OK;
}

// ---------------------------------------------------------------------------
// Mixed precision: block column by the float recursion, refined in FP64.
// A single call is a batch of one.
// ---------------------------------------------------------------------------
struct RefineCache {
  std::shared_ptr<CachedPlan> col, sol;
  std::vector<int> kept;
  bool column_gives_x0 = true;
};

typedef std::tuple<int64_t, int, int, int, int> RefineKey;  // n, k, j, width, reuse

// Outcome of the calling thread's last mixed-precision call.
thread_local int t_last_sweeps = 0;
thread_local double t_last_update = 0.0;
thread_local int t_last_range_fallback = 0;  // FP16 products redone in BF16

std::shared_ptr<RefineCache> get_refine(int64_t n, int k, int j, int width, int reuse) {
  static std::map<RefineKey, std::shared_ptr<RefineCache>> c;
  RefineKey key(n, k, j, width, reuse);
  std::lock_guard<std::mutex> g(g_cache_mu);
  auto itp = c.find(key);
  if (itp != c.end()) return itp->second;
  RefinePlans rp = make_refine_plans(n, k, j, width, reuse != 0);
  auto rc = std::make_shared<RefineCache>();
  rc->col = std::make_shared<CachedPlan>();
  rc->sol = std::make_shared<CachedPlan>();
  rc->col->plan = std::move(rp.column);
  rc->sol->plan = std::move(rp.solve);
  rc->col->layout = make_layout(rc->col->plan, 4);
  rc->sol->layout = make_layout(rc->sol->plan, 4);
  rc->kept = rp.kept;
  rc->column_gives_x0 = rp.column_gives_x0;
  if (c.size() > 1024) c.clear();
  c[key] = rc;
  return rc;
}

// Per-problem buffers of the mixed path (offsets inside the problem's region).
struct MixedRegion {
  size_t x64 = 0, r64 = 0, r32 = 0, d32 = 0, plans = 0, total = 0;
};

MixedRegion mixed_region(int64_t n, int k, const RefineCache& rc) {
  MixedRegion L;
  const size_t b = static_cast<size_t>((n + k - 1) / k);
  const size_t kb = static_cast<size_t>(k) * b;
  size_t off = 0;
  L.x64 = off;
  off += align_up(kb * b * 8);
  L.r64 = off;
  off += align_up(kb * b * 8);
  L.r32 = off;
  off += align_up(kb * b * 4);
  L.d32 = off;
  off += align_up(kb * b * 4);
  L.plans = off;
  off += align_up(std::max(rc.col->layout.desc_off, rc.sol->layout.desc_off));  // slots of both plans
  L.total = off;
  return L;
}

// Workspace of a mixed call over count problems: the problems' regions, then
// shared: status word, device scalars (kRefineScalars per problem),
// refinement items, residual product items, output copy items, merged
// descriptors of the block-column plans and of the correction solves.
struct MixedBatch {
  std::vector<std::shared_ptr<RefineCache>> rc;
  std::vector<MixedRegion> reg;
  std::vector<size_t> region;
  MergedLayout col, sol;
  size_t info_off = 0, flag_off = 0, scal_off = 0, items_off = 0, gemm_off = 0, load_off = 0, col_off = 0, sol_off = 0;
  size_t split_off = 0, split_bytes = 0;
  size_t desc_bytes = 0, total = 0;
};

// Scratch of the split products (mixed FP16 and BF16): room for the split
// operands (three BF16 planes, which an FP16 call needs when it falls back
// to BF16) of the largest explicit product step of the merged plans, at
// most kSplitCap bytes (larger steps run in parts).
constexpr size_t kSplitCap = size_t(2) << 30;
size_t split_scratch_bytes(const std::vector<const Plan*>& plans, const MergedLayout& m, int precision) {
  if (precision != BRI_MIXED_F16 && precision != BRI_MIXED_BF16) return 0;
  int bmax = 0;
  for (const Plan* p : plans) bmax = std::max(bmax, p->b);
  size_t items = 0;
  for (const std::vector<int>& g : m.groups) {
    const Plan& p0 = *plans[g[0]];
    for (size_t si = 0; si < p0.steps.size(); ++si) {
      const StepKind kd = p0.steps[si].kind;
      if (kd == ST_LOAD || kd == ST_GETRF || kd == ST_TRTRI) continue;
      size_t n = 0;
      for (int t : g) n += plans[t]->steps[si].items.size();
      items = std::max(items, n);
    }
  }
  const size_t per = static_cast<size_t>(split_item_bytes(bmax, bmax, split_pitch(bmax), 3));
  return align_up(std::min(kSplitCap, items * per));
}

MixedBatch make_mixed_batch(int count, const int64_t* n, const int* k, const int* j, const bri_opts* o,
                            bool merged_width_rule) {
  MixedBatch mb;
  mb.rc.resize(count);
  mb.reg.resize(count);
  mb.region.resize(count);
  std::vector<const Plan*> pc(count), ps(count);
  size_t off = 0;
  for (int t = 0; t < count; ++t) {
    const int w = merged_width_rule ? merged_width(k[t]) : resolve_width(n[t], k[t], o);
    mb.rc[t] = get_refine(n[t], k[t], j[t], w, o->reuse);
    mb.reg[t] = mixed_region(n[t], k[t], *mb.rc[t]);
    mb.region[t] = off;
    off += mb.reg[t].total;
    pc[t] = &mb.rc[t]->col->plan;
    ps[t] = &mb.rc[t]->sol->plan;
  }
  mb.col = merge_layout(pc);
  mb.sol = merge_layout(ps);
  mb.info_off = off;  // a status word per problem (when the caller passes no d_info)
  off += align_up(sizeof(int32_t) * count);
  mb.flag_off = off;  // FP16 range flag
  off += kAlign;
  const size_t c = static_cast<size_t>(count);
  mb.scal_off = off;
  off += align_up(c * kRefineScalars * sizeof(double));
  // descriptors, uploaded with one copy
  const size_t d0 = off;
  mb.items_off = off;
  off += align_up(c * sizeof(RefItem));
  mb.gemm_off = off;
  off += align_up(c * sizeof(GemmItem));
  mb.load_off = off;
  off += align_up(c * sizeof(LoadItem));
  mb.col_off = off;
  off += mb.col.bytes;
  mb.sol_off = off;
  off += mb.sol.bytes;
  mb.desc_bytes = off - d0;
  // Split scratch last, within a sixteenth of the rest (so that narrow
  // widths under a memory budget stay lean; larger steps run in parts).
  const size_t want = std::max(split_scratch_bytes(pc, mb.col, o->precision), split_scratch_bytes(ps, mb.sol, o->precision));
  mb.split_off = off;
  mb.split_bytes = std::min(want, off / 16 / kAlign * kAlign);
  off += mb.split_bytes;
  mb.total = off;
  return mb;
}

size_t mixed_workspace_size(int64_t n, int k, int j, const bri_opts* o) {
  return make_mixed_batch(1, &n, &k, &j, o, false).total;
}

int run_mixed_batch(const MixedBatch& mb, int count, const void* const* M, const int64_t* n, const int64_t* ldm,
                    const int* i, const int* j, void* const* out, const int64_t* ldo, const bri_opts* o) {
  hipStream_t st = o->stream;
  char* ws = static_cast<char*>(o->workspace);
  int32_t* info_words = o->d_info ? o->d_info : reinterpret_cast<int32_t*>(ws + mb.info_off);
  double* scal_all = reinterpret_cast<double*>(ws + mb.scal_off);
  const size_t d0 = mb.items_off;
  std::vector<Ctx> cc(count), cs(count);
  std::vector<const Plan*> pc(count), ps(count);
  std::vector<RefItem> ri(count);
  std::vector<GemmItem> gi(count);
  std::vector<LoadItem> li(count);
  int64_t max_nn = 0, max_kb_b = 0, max_fix = 0;
  int max_n = 0, max_b = 0;
  for (int t = 0; t < count; ++t) {
    const RefineCache& rc = *mb.rc[t];
    const MixedRegion& R = mb.reg[t];
    char* base = ws + mb.region[t];
    const int b = rc.col->plan.b;
    const int64_t kb = static_cast<int64_t>(rc.col->plan.k) * b;
    RefItem& r = ri[t];
    std::memset(&r, 0, sizeof(r));
    r.M = static_cast<const double*>(M[t]);
    r.n = n[t];
    r.ldm = ldm[t];
    r.kb = kb;
    r.b = b;
    r.j = j[t];
    r.X = reinterpret_cast<double*>(base + R.x64);
    r.R = reinterpret_cast<double*>(base + R.r64);
    r.R32 = reinterpret_cast<float*>(base + R.r32);
    r.D = reinterpret_cast<float*>(base + R.d32);
    r.scal = scal_all + static_cast<size_t>(t) * kRefineScalars;
    max_nn = std::max<int64_t>(max_nn, n[t] * n[t]);
    max_kb_b = std::max<int64_t>(max_kb_b, kb * b);
    max_fix = std::max<int64_t>(max_fix, static_cast<int64_t>(b) * (1 + kb - n[t]));
    max_n = std::max<int>(max_n, static_cast<int>(n[t]));
    max_b = std::max(max_b, b);
    // R[0:n) = -M X[0:n) in FP64
    GemmItem& g = gi[t];
    std::memset(&g, 0, sizeof(g));
    g.A = g.B = g.Cin = g.Sub = zero_view();
    g.A.p = M[t];
    g.A.ld = ldm[t];
    g.A.rows = static_cast<int32_t>(n[t]);
    g.A.cols = static_cast<int32_t>(n[t]);
    g.B.p = r.X;
    g.B.ld = b;
    g.B.rows = static_cast<int32_t>(kb);
    g.B.cols = b;
    g.out = r.R;
    g.ldo = b;
    g.M = static_cast<int32_t>(n[t]);
    g.N = b;
    g.K = static_cast<int32_t>(n[t]);
    g.alpha = -1.0;
    // block row i of X to out
    LoadItem& l = li[t];
    std::memset(&l, 0, sizeof(l));
    l.src = zero_view();
    l.src.p = r.X + static_cast<int64_t>(i[t]) * b * b;
    l.src.ld = b;
    l.src.rows = b;
    l.src.cols = b;
    l.dst = out[t];
    l.ldd = ldo[t];
    l.rows = b;
    l.cols = b;
    // float plans: blocks of sigma Gamma loaded from M (converted and scaled
    // by the load steps), D as the output, R32 as the right-hand side
    Ctx& c = cc[t];
    c.pivoting = o->pivoting;
    c.lu = o->factorization;
    c.M = static_cast<const char*>(M[t]);
    c.n = n[t];
    c.ldm = ldm[t];
    c.m_elem = 8;
    c.m_max = r.scal;  // scal[0]: max |M|
    c.b = b;
    c.elem = 4;
    c.ws = base + R.plans;
    c.lay = &rc.col->layout;
    c.out = reinterpret_cast<char*>(r.D);
    c.ldo = b;
    c.info = info_words + t;
    c.rhs = reinterpret_cast<char*>(r.R32);
    c.ldr = b;
    c.lp = lp_of(o->precision);
    cs[t] = c;
    cs[t].lay = &rc.sol->layout;
    pc[t] = &rc.col->plan;
    ps[t] = &rc.sol->plan;
  }
  // Panel pivoting kernels take one block order per launch: merged groups
  // must then hold one order only (single calls always do).
  Staging& sg = staging();
  std::lock_guard<std::mutex> lk(sg.mu);
  char* host = sg.get(mb.desc_bytes);
  if (!host) return BRI_ERR_HIP;
  std::memcpy(host + (mb.items_off - d0), ri.data(), count * sizeof(RefItem));
  std::memcpy(host + (mb.gemm_off - d0), gi.data(), count * sizeof(GemmItem));
  int ndl_resid = count;
  for (const GemmItem& g : gi)
    if (!gemm_item_is_direct(g, 8)) ndl_resid = 0;
  std::memcpy(host + (mb.load_off - d0), li.data(), count * sizeof(LoadItem));
  MergedExec ecol, esol;
  try {
    ecol = merge_write(pc, cc, mb.col, host + (mb.col_off - d0), ws + mb.col_off);
    esol = merge_write(ps, cs, mb.sol, host + (mb.sol_off - d0), ws + mb.sol_off);
  } catch (const std::exception&) {
    return BRI_ERR_UNSUPPORTED;
  }
  if (o->pivoting == BRI_PIVOT_PANEL) {
    for (const MergedExec* e : {&ecol, &esol})
      for (size_t g = 0; g < e->groups.size(); ++g)
        for (int t : (e == &ecol ? mb.col : mb.sol).groups[g])
          if (cc[t].b != e->bmax[g]) return BRI_ERR_UNSUPPORTED;
  }
  if (hipMemcpyAsync(ws + d0, host, mb.desc_bytes, hipMemcpyHostToDevice, st) != hipSuccess) return BRI_ERR_HIP;
  if (hipEventRecord(sg.ev, st) != hipSuccess) return BRI_ERR_HIP;
  const RefItem* d_items = reinterpret_cast<const RefItem*>(ws + mb.items_off);
  if (launch_fill_int(info_words, count, 0, st) != hipSuccess) return BRI_ERR_HIP;

  // Float recursion: products per the precision, tile factorisations in FP64.
  // The FP16 split products flag operand values outside the FP16 range; the
  // call then starts again with the BF16 split products (same exponent range
  // as FP32), found at the first sweep's synchronisation.
  int32_t* range_flag = reinterpret_cast<int32_t*>(ws + mb.flag_off);
  ExecCfg mcfg{o->pivoting, o->factorization, lp_of(o->precision), true, range_flag,
               mb.split_bytes ? ws + mb.split_off : nullptr, mb.split_bytes,
               count == 1 ? reinterpret_cast<unsigned long long*>(o->d_stats) : nullptr, ws, o->workspace_bytes};
  t_last_range_fallback = 0;
  std::vector<char> conv;
  std::vector<double> prev;
  std::vector<double> hs(static_cast<size_t>(count) * kRefineScalars);
  for (int pass = 0;; ++pass) {
  if (mcfg.lp == 1 && launch_fill_int(range_flag, 1, 0, st) != hipSuccess) return BRI_ERR_HIP;
  if (mcfg.stats && launch_fill_int(reinterpret_cast<int32_t*>(mcfg.stats), 8, 0, st) != hipSuccess)
    return BRI_ERR_HIP;
  // sigma from max |M|, then X0 = sigma (sigma Gamma)^{-1} E_j by the float
  // block-column plans (which keep their pivots for the correction solves).
  if (launch_scal_clear(d_items, count, 0, kRefineScalars, st) != hipSuccess) return BRI_ERR_HIP;
  if (launch_absmax(d_items, count, 0, max_nn, st) != hipSuccess) return BRI_ERR_HIP;
  int rcode = run_merged<float>(ecol, mcfg, st);
  if (rcode != BRI_OK) return rcode;
  if (!mb.rc[0]->column_gives_x0) {
    // Pivots only (reuse): X0 = (sigma Gamma)^{-1} E_j by the solve plan.
    if (launch_set_ej(d_items, count, max_kb_b, st) != hipSuccess) return BRI_ERR_HIP;
    rcode = run_merged<float>(esol, mcfg, st);
    if (rcode != BRI_OK) return rcode;
  }
  if (launch_refine_update(d_items, count, max_kb_b, 1, st) != hipSuccess) return BRI_ERR_HIP;

  // Sweeps: R = E_j - Gamma X (FP64), D = (sigma Gamma)^{-1} (s R) by the float
  // solves, X += (sigma / s) D.  A problem has converged when its correction
  // is below tol ||X||_F, or, from the second sweep on, when the observed
  // contraction rho = ||dX_t|| / ||dX_{t-1}|| < 1/2 bounds the remaining
  // error rho / (1 - rho) ||dX_t|| below it.  All problems sweep together
  // until every one has converged.
  conv.assign(count, o->refine_max_iters <= 0 ? 1 : 0);
  prev.assign(count, 0.0);
  const double tol = o->refine_tol;
  t_last_sweeps = 0;
  t_last_update = 0.0;
  bool restart = false;
  for (int it = 0; it < std::max(1, o->refine_max_iters); ++it) {
    if (o->refine_max_iters <= 0) {
      // no sweeps: only the range check of the FP16 products
      if (mcfg.lp != 1) break;
      int32_t hf = 0;
      if (hipMemcpyAsync(&hf, range_flag, sizeof(hf), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return BRI_ERR_HIP;
      restart = hf != 0;
      break;
    }
    if (launch_scal_clear(d_items, count, 1, 4, st) != hipSuccess) return BRI_ERR_HIP;
    GemmLaunch L{};
    L.mode = GEMM_EXPLICIT;
    L.elem = 8;
    L.items = ws + mb.gemm_off;
    L.count = count;
    L.w = count;        // stored dense operands
    L.ndl = ndl_resid;  // all of them for the direct-to-LDS instance when they qualify
    if (launch_gemm<double>(L, max_n, max_b, st) != hipSuccess) return BRI_ERR_HIP;
    if (launch_resid_fix(d_items, count, max_fix, st) != hipSuccess) return BRI_ERR_HIP;
    if (launch_absmax(d_items, count, 1, max_kb_b, st) != hipSuccess) return BRI_ERR_HIP;
    if (launch_rhs_scale(d_items, count, max_kb_b, st) != hipSuccess) return BRI_ERR_HIP;
    rcode = run_merged<float>(esol, mcfg, st);
    if (rcode != BRI_OK) return rcode;
    if (launch_refine_update(d_items, count, max_kb_b, 0, st) != hipSuccess) return BRI_ERR_HIP;
    if (hipMemcpyAsync(hs.data(), scal_all, hs.size() * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
      return BRI_ERR_HIP;
    int32_t hflag = 0;
    if (mcfg.lp == 1 && it == 0 &&
        hipMemcpyAsync(&hflag, range_flag, sizeof(hflag), hipMemcpyDeviceToHost, st) != hipSuccess)
      return BRI_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return BRI_ERR_HIP;
    if (hflag) {
      restart = true;
      break;
    }
    t_last_sweeps = it + 1;
    bool all = true;
    double worst = 0.0;
    for (int t = 0; t < count; ++t) {
      const double dd = hs[static_cast<size_t>(t) * kRefineScalars + 2];
      const double xx = hs[static_cast<size_t>(t) * kRefineScalars + 3];
      const double upd = std::sqrt(dd), lim = tol * std::sqrt(xx);
      worst = std::max(worst, xx > 0 ? upd / std::sqrt(xx) : upd);
      if (!conv[t] && std::isfinite(dd) && std::isfinite(xx)) {
        bool done = upd <= lim;
        if (!done && prev[t] > 0) {
          const double rho = upd / prev[t];
          done = rho < 0.5 && rho / (1.0 - rho) * upd <= lim;
        }
        if (done) conv[t] = 1;
      }
      prev[t] = upd;
      all = all && conv[t];
    }
    t_last_update = worst;
    if (all) break;
  }
  if (!restart) break;
  mcfg.lp = 2;
  t_last_range_fallback = 1;
  }  // passes
  if (launch_load<double>(reinterpret_cast<const LoadItem*>(ws + mb.load_off), count, max_b, max_b, st) !=
      hipSuccess)
    return BRI_ERR_HIP;
  for (int t = 0; t < count; ++t)
    if (!conv[t] && launch_info_unconverged(info_words + t, st) != hipSuccess)
      return BRI_ERR_HIP;
  return BRI_OK;
}

int invert_block_mixed(const void* M, int64_t n, int64_t ldm, int k, int i, int j, void* out, int64_t ldo,
                       const bri_opts* o) {
  MixedBatch mb;
  try {
    mb = make_mixed_batch(1, &n, &k, &j, o, false);
  } catch (const std::exception&) {
    return BRI_ERR_UNSUPPORTED;
  }
  if (!o->workspace || o->workspace_bytes < mb.total) return BRI_ERR_WORKSPACE;
  return run_mixed_batch(mb, 1, &M, &n, &ldm, &i, &j, &out, &ldo, o);
}

}  // namespace
}  // namespace bri

using namespace bri;

extern "C" {

void bri_default_opts(bri_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = BRI_F64;
  o->concurrency = 0;
  o->pivoting = BRI_PIVOT_AUTO;
  o->refine_max_iters = 10;
  o->refine_tol = 1e-12;
}

const char* bri_version(void) { return "bri-mi355x 0.1"; }

size_t bri_opts_size(void) { return sizeof(bri_opts); }

const char* bri_status_string(int status) {
  if (status == BRI_OK) return "success";
  if (status == BRI_ERR_HIP) return "HIP launch or copy failed";
  if (status == BRI_ERR_WORKSPACE) return "workspace smaller than required";
  if (status == BRI_ERR_UNSUPPORTED) return "size or precision not supported";
  if (status < 0 && status > -100) return "invalid argument (see the position -status)";
  return "unknown status";
}

static int check_block_args(int64_t n, int64_t ldm, int k, int i, int j, int64_t ldo) {
  if (n < 1) return -2;
  if (ldm < n) return -3;
  if (k < 2 || k > n) return -4;
  if (i < 0 || i >= k) return -5;
  if (j < 0 || j >= k) return -6;
  const int64_t b = (n + k - 1) / k;
  if (ldo < b) return -8;
  if (b > BRI_MAX_BLOCK) return BRI_ERR_UNSUPPORTED;
  return 0;
}

int bri_refine_last(int* sweeps, double* last_update, int* bf16_fallback) {
  if (sweeps) *sweeps = t_last_sweeps;
  if (last_update) *last_update = t_last_update;
  if (bf16_fallback) *bf16_fallback = t_last_range_fallback;
  return 0;
}

int bri_profile_enable(int on) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  const int was = g_prof_on ? 1 : 0;
  g_prof_on = on != 0;
  return was;
}

int bri_profile_read(bri_profile_entry* entries, int cap) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  for (ProfRecord& r : g_prof_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.e1) != hipSuccess || hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess)
      return BRI_ERR_HIP;
    bri_profile_entry& e = g_prof_acc[r.kind];
    e.steps += 1;
    e.launches += r.launches;
    e.ms += ms;
    e.flops += r.flops;
    g_prof_pool.push_back(r.e0);
    g_prof_pool.push_back(r.e1);
  }
  g_prof_pending.clear();
  const int n = std::min(cap, BRI_PROFILE_KINDS);
  for (int t = 0; t < n; ++t) entries[t] = g_prof_acc[t];
  std::memset(g_prof_acc, 0, sizeof(g_prof_acc));
  return n;
}

static size_t workspace_size_of(int64_t n, int k, int i, int j, const bri_opts* o) {
  if (!order_ok(o)) return 0;
  const int w = resolve_width(n, k, o);
  if (mixed_precision(o->precision)) {
    try {
      return mixed_workspace_size(n, k, j, o);
    } catch (const std::exception&) {
      return 0;
    }
  }
  if (!plain_precision(o->precision)) return 0;
  try {
    auto cp = get_plan(block_kind(o), n, k, i, j, w, elem_size(o->precision), 0);
    return cp->layout.total;
  } catch (const std::exception&) {
    return 0;
  }
}

// The status word a single invert_block call uses when the caller passes no
// d_info (inside the workspace), or null when the workspace is too small.
static int32_t* block_info_word(int64_t n, int k, int i, int j, const bri_opts* o) {
  try {
    size_t off = 0, need = 0;
    if (mixed_precision(o->precision)) {
      const MixedBatch mb = make_mixed_batch(1, &n, &k, &j, o, false);
      off = mb.info_off;
      need = mb.total;
    } else {
      auto cp = get_plan(block_kind(o), n, k, i, j, resolve_width(n, k, o), elem_size(o->precision), 0);
      off = cp->layout.info_off;
      need = cp->layout.total;
    }
    if (!o->workspace || o->workspace_bytes < need) return nullptr;
    return reinterpret_cast<int32_t*>(static_cast<char*>(o->workspace) + off);
  } catch (const std::exception&) {
    return nullptr;
  }
}

static bri_opts block_budget(const bri_opts* o, int64_t n, int k, int i, int j, bool& fits) {
  return with_budget(o, n, k, [&](const bri_opts& r) { return workspace_size_of(n, k, i, j, &r); }, fits);
}

size_t bri_workspace_size(int64_t n, int k, int i, int j, const bri_opts* o) {
  if (!o || check_block_args(n, n, k, i, j, (n + k - 1) / k) != 0) return 0;
  bool fits;
  const bri_opts ob = block_budget(o, n, k, i, j, fits);
  return fits ? workspace_size_of(n, k, i, j, &ob) : 0;
}

int bri_plan_describe(int64_t n, int k, int i, int j, const bri_opts* o, bri_plan_stats* s) {
  if (!s) return -6;
  if (!o) return -5;
  const int rc = check_block_args(n, n, k, i, j, (n + k - 1) / k);
  if (rc) return rc;
  bool fits;
  const bri_opts ob = block_budget(o, n, k, i, j, fits);
  if (!fits) return BRI_ERR_WORKSPACE;
  o = &ob;
  if (!order_ok(o)) return BRI_ERR_UNSUPPORTED;
  const int w = resolve_width(n, k, o);
  auto cp = get_plan(block_kind(o), n, k, i, j, w, elem_size(o->precision), 0);
  const Plan& p = cp->plan;
  s->schur_ops = p.schur_ops;
  s->final_inversions = p.final_inversions;
  s->slots = p.nslots;
  s->batch_width = p.width;
  s->steps = static_cast<int64_t>(p.steps.size());
  int64_t launches = 1;  // clearing d_info
  for (const Step& st : p.steps)
    launches += step_launches(st.kind, static_cast<int>(st.items.size()), p.b, o->pivoting, true, o->factorization);
  s->kernel_launches = launches;
  s->block = p.b;
  s->algorithmic_flops = p.algorithmic_flops;
  s->executed_flops = p.executed_flops;
  s->workspace_bytes = mixed_precision(o->precision) ? mixed_workspace_size(n, k, j, o) : cp->layout.total;
  return 0;
}

}  // extern "C"

namespace {
int64_t dump_steps(const Plan& plan, int64_t* words, int64_t cap) {
  int64_t pos = 0;
  auto put = [&](int64_t v) {
    if (words && pos < cap) words[pos] = v;
    ++pos;
  };
  auto opnd = [&](const Opnd& x) {
    put(x.kind);
    put(x.a);
    put(x.b);
  };
  for (const Step& s : plan.steps) {
    put(s.kind);
    put(static_cast<int64_t>(s.items.size()));
    for (const StepItem& it : s.items) {
      opnd(it.dst);
      opnd(it.x);
      opnd(it.y);
      opnd(it.cin);
      opnd(it.sub);
      put(it.node);
    }
  }
  return pos;
}
}  // namespace

extern "C" {

int64_t bri_plan_dump(int64_t n, int k, int i, int j, const bri_opts* o, int64_t* words, int64_t cap) {
  if (!o) return -5;
  const int rc = check_block_args(n, n, k, i, j, (n + k - 1) / k);
  if (rc) return rc;
  if (!order_ok(o)) return BRI_ERR_UNSUPPORTED;
  const int w = resolve_width(n, k, o);
  auto cp = get_plan(block_kind(o), n, k, i, j, w, elem_size(o->precision), 0);
  return dump_steps(cp->plan, words, cap);
}

int64_t bri_refine_plan_dump(int64_t n, int k, int j, int which, const bri_opts* o, int64_t* words, int64_t cap) {
  if (!o) return -5;
  const int rc = check_block_args(n, n, k, 0, j, (n + k - 1) / k);
  if (rc) return rc == -6 ? -3 : rc;
  if (which < 0 || which > 2) return -4;
  const int w = resolve_width(n, k, o);
  auto r = get_refine(n, k, j, w, o->reuse);
  if (which == 2) {
    for (int t = 0; t < k; ++t)
      if (words && t < cap) words[t] = r->kept[t];
    return k;
  }
  return dump_steps(which == 0 ? r->col->plan : r->sol->plan, words, cap);
}

}  // extern "C"

// invert_block; noalloc: the workspace is the caller's scratch and the
// descriptors are staged without allocating (invert_block_noalloc).
static int invert_block_impl(const void* M, int64_t n, int64_t ldm, int k, int i, int j, void* out, int64_t ldo,
                             const bri_opts* o, bool noalloc) {
  if (!M) return -1;
  if (!out) return -7;
  if (!o) return -9;
  const int rc = check_block_args(n, ldm, k, i, j, ldo);
  if (rc) return rc;
  bool fits;
  const bri_opts ob = block_budget(o, n, k, i, j, fits);
  if (!fits) return BRI_ERR_WORKSPACE;
  o = &ob;
  if (!order_ok(o)) return BRI_ERR_UNSUPPORTED;
  if (o->pivoting == BRI_PIVOT_AUTO) {
    // Tile pivoting first; if a factorisation reported a failed pivot or
    // element growth, the block again with panel pivoting.
    bri_opts t = *o;
    t.pivoting = BRI_PIVOT_TILE;
    if (!t.d_info) {
      t.d_info = block_info_word(n, k, i, j, o);
      if (!t.d_info) return BRI_ERR_WORKSPACE;
    }
    int rc2 = invert_block_impl(M, n, ldm, k, i, j, out, ldo, &t, noalloc);
    int32_t h = 0;
    if (rc2 == BRI_OK) rc2 = read_info1(t.d_info, h, o->stream);
    if (rc2 != BRI_OK || h <= 0) return rc2;
    t.pivoting = BRI_PIVOT_PANEL;
    return invert_block_impl(M, n, ldm, k, i, j, out, ldo, &t, noalloc);
  }
  if (mixed_precision(o->precision)) {
    if (noalloc) return BRI_ERR_UNSUPPORTED;
    return invert_block_mixed(M, n, ldm, k, i, j, out, ldo, o);
  }
  if (!plain_precision(o->precision)) return BRI_ERR_UNSUPPORTED;
  const int elem = elem_size(o->precision);
  const int w = resolve_width(n, k, o);
  std::shared_ptr<CachedPlan> cp;
  try {
    cp = get_plan(block_kind(o), n, k, i, j, w, elem, 0);
  } catch (const std::exception&) {
    return BRI_ERR_UNSUPPORTED;
  }
  if (!o->workspace || o->workspace_bytes < cp->layout.total) return BRI_ERR_WORKSPACE;
  Ctx c;
  c.pivoting = o->pivoting;
  c.lu = o->factorization;
  c.M = static_cast<const char*>(M);
  c.n = n;
  c.ldm = ldm;
  c.b = cp->plan.b;
  c.elem = elem;
  c.ws = static_cast<char*>(o->workspace);
  c.out = static_cast<char*>(out);
  c.ldo = ldo;
  c.info = o->d_info ? o->d_info : reinterpret_cast<int32_t*>(c.ws + cp->layout.info_off);
  c.stats = reinterpret_cast<unsigned long long*>(o->d_stats);
  c.stats_base = static_cast<const char*>(o->workspace);
  c.stats_limit = o->workspace_bytes;
  return execute(*cp, c, o->stream, true, noalloc);
}

namespace bri {
int invert_block_scratch(const void* M, int64_t n, int64_t ldm, int k, int i, int j, void* out, int64_t ldo,
                         const bri_opts* o, void* scratch, size_t scratch_bytes) {
  if (!o) return -9;
  bri_opts t = *o;
  t.workspace = scratch;
  t.workspace_bytes = scratch_bytes;
  if (t.concurrency <= 0) t.workspace_budget = scratch_bytes;  // the widest width that fits
  return invert_block_impl(M, n, ldm, k, i, j, out, ldo, &t, true);
}
}  // namespace bri

extern "C" {

int invert_block(const void* M, int64_t n, int64_t ldm, int k, int i, int j, void* out, int64_t ldo,
                 const bri_opts* o) {
  return invert_block_impl(M, n, ldm, k, i, j, out, ldo, o, false);
}

static size_t column_size_of(int64_t n, int k, int j, const bri_opts* o) {
  const int w = resolve_width(n, k, o);
  try {
    auto cp = get_plan(1, n, k, 0, j, w, elem_size(o->precision), 0);
    return cp->layout.total;
  } catch (const std::exception&) {
    return 0;
  }
}

static bri_opts column_budget(const bri_opts* o, int64_t n, int k, int j, bool& fits) {
  return with_budget(o, n, k, [&](const bri_opts& r) { return column_size_of(n, k, j, &r); }, fits);
}

size_t bri_block_column_workspace_size(int64_t n, int k, int j, const bri_opts* o) {
  if (!o || check_block_args(n, n, k, 0, j, (n + k - 1) / k) != 0) return 0;
  if (!plain_precision(o->precision)) return 0;
  bool fits;
  const bri_opts ob = column_budget(o, n, k, j, fits);
  return fits ? column_size_of(n, k, j, &ob) : 0;
}

int bri_block_column(const void* M, int64_t n, int64_t ldm, int k, int j, int transpose, void* X, int64_t ldx,
                     const bri_opts* o) {
  if (!M) return -1;
  if (!X) return -7;
  if (!o) return -9;
  if (o->order != BRI_ORDER_PRINCIPAL) return BRI_ERR_UNSUPPORTED;  // the column plan is principal
  const int rc = check_block_args(n, ldm, k, 0, j, ldx);
  if (rc) return rc == -8 ? -8 : (rc == -6 ? -5 : rc);
  if (!plain_precision(o->precision)) return BRI_ERR_UNSUPPORTED;
  bool fits;
  const bri_opts ob = column_budget(o, n, k, j, fits);
  if (!fits) return BRI_ERR_WORKSPACE;
  o = &ob;
  if (o->pivoting == BRI_PIVOT_AUTO) {
    bri_opts t = *o;
    t.pivoting = BRI_PIVOT_TILE;
    if (!t.d_info) {
      std::shared_ptr<CachedPlan> cp;
      try {
        cp = get_plan(1, n, k, 0, j, resolve_width(n, k, o), elem_size(o->precision), transpose ? 1 : 0);
      } catch (const std::exception&) {
        return BRI_ERR_UNSUPPORTED;
      }
      if (!o->workspace || o->workspace_bytes < cp->layout.total) return BRI_ERR_WORKSPACE;
      t.d_info = reinterpret_cast<int32_t*>(static_cast<char*>(o->workspace) + cp->layout.info_off);
    }
    int rc2 = bri_block_column(M, n, ldm, k, j, transpose, X, ldx, &t);
    std::vector<int32_t> h;
    if (rc2 == BRI_OK) rc2 = read_info(t.d_info, 1, h, o->stream);
    if (rc2 != BRI_OK || h[0] <= 0) return rc2;
    t.pivoting = BRI_PIVOT_PANEL;
    return bri_block_column(M, n, ldm, k, j, transpose, X, ldx, &t);
  }
  const int elem = elem_size(o->precision);
  const int w = resolve_width(n, k, o);
  std::shared_ptr<CachedPlan> cp;
  try {
    cp = get_plan(1, n, k, 0, j, w, elem, transpose ? 1 : 0);
  } catch (const std::exception&) {
    return BRI_ERR_UNSUPPORTED;
  }
  if (!o->workspace || o->workspace_bytes < cp->layout.total) return BRI_ERR_WORKSPACE;
  Ctx c;
  c.pivoting = o->pivoting;
  c.lu = o->factorization;
  c.M = static_cast<const char*>(M);
  c.n = n;
  c.ldm = ldm;
  c.b = cp->plan.b;
  c.elem = elem;
  c.transpose = transpose ? 1 : 0;
  c.ws = static_cast<char*>(o->workspace);
  c.out = static_cast<char*>(X);
  c.ldo = ldx;
  c.info = o->d_info ? o->d_info : reinterpret_cast<int32_t*>(c.ws + cp->layout.info_off);
  return execute(*cp, c, o->stream, true);
}

static int check_batch_args(int count, const int64_t* n, const int* k, const int* i, const int* j) {
  for (int t = 0; t < count; ++t) {
    const int rc = check_block_args(n[t], n[t], k[t], i[t], j[t], (n[t] + k[t] - 1) / k[t]);
    if (rc) return rc;
  }
  return 0;
}

size_t bri_batched_workspace_size(int count, const int64_t* n, const int* k, const int* i, const int* j,
                                  const bri_opts* o) {
  if (count < 0 || !n || !k || !i || !j || !o) return 0;
  if (o->order != BRI_ORDER_PRINCIPAL) return 0;
  if (check_batch_args(count, n, k, i, j) != 0) return 0;
  if (count == 0) return kAlign;
  if (batch_mergeable(o)) {
    try {
      return mixed_precision(o->precision) ? make_mixed_batch(count, n, k, j, o, true).total
                                           : make_batch_plan(count, n, k, i, j, elem_size(o->precision), o->reuse).total;
    } catch (const std::exception&) {
      return 0;
    }
  }
  size_t m = 0;
  for (int t = 0; t < count; ++t) {
    const size_t s = bri_workspace_size(n[t], k[t], i[t], j[t], o);
    if (s == 0) return 0;
    m = std::max(m, s);
  }
  return m;
}

int invert_block_batched(int count, const void* const* M, const int64_t* n, const int64_t* ldm, const int* k,
                         const int* i, const int* j, void* const* out, const int64_t* ldo, const bri_opts* o) {
  if (count < 0) return -1;
  if (!M) return -2;
  if (!n) return -3;
  if (!ldm) return -4;
  if (!k) return -5;
  if (!i) return -6;
  if (!j) return -7;
  if (!out) return -8;
  if (!ldo) return -9;
  if (!o) return -10;
  if (o->order != BRI_ORDER_PRINCIPAL) return BRI_ERR_UNSUPPORTED;
  if (count == 0) return BRI_OK;
  for (int t = 0; t < count; ++t) {
    if (!M[t]) return -2;
    if (!out[t]) return -8;
    const int rc = check_block_args(n[t], ldm[t], k[t], i[t], j[t], ldo[t]);
    if (rc) return rc == -2 ? -3 : rc == -3 ? -4 : rc == -4 ? -5 : rc == -5 ? -6 : rc == -6 ? -7 : rc == -8 ? -9 : rc;
  }
  if (o->pivoting == BRI_PIVOT_AUTO && batch_mergeable(o)) {
    // Merged tile-pivoting pass; problems whose factorisations reported a
    // failed pivot or element growth are then computed again one by one with
    // panel pivoting in the same workspace.
    bri_opts t = *o;
    t.pivoting = BRI_PIVOT_TILE;
    if (!t.d_info) {
      size_t off = 0, need = 0;
      try {
        if (mixed_precision(o->precision)) {
          const MixedBatch mb = make_mixed_batch(count, n, k, j, o, true);
          off = mb.info_off;
          need = mb.total;
        } else {
          const BatchPlan bp = make_batch_plan(count, n, k, i, j, elem_size(o->precision), o->reuse);
          off = bp.info_off;
          need = bp.total;
        }
      } catch (const std::exception&) {
        return BRI_ERR_UNSUPPORTED;
      }
      if (!o->workspace || o->workspace_bytes < need) return BRI_ERR_WORKSPACE;
      t.d_info = reinterpret_cast<int32_t*>(static_cast<char*>(o->workspace) + off);
    }
    int rc2 = invert_block_batched(count, M, n, ldm, k, i, j, out, ldo, &t);
    std::vector<int32_t> h;
    if (rc2 == BRI_OK) rc2 = read_info(t.d_info, count, h, o->stream);
    if (rc2 != BRI_OK) return rc2;
    for (int p = 0; p < count; ++p) {
      if (h[p] <= 0) continue;
      bri_opts tt = *o;
      tt.pivoting = BRI_PIVOT_PANEL;
      tt.concurrency = 0;
      tt.workspace_budget = o->workspace_bytes;
      tt.d_info = o->d_info ? o->d_info + p : nullptr;
      rc2 = invert_block(M[p], n[p], ldm[p], k[p], i[p], j[p], out[p], ldo[p], &tt);
      if (rc2 != BRI_OK && rc2 != BRI_ERR_WORKSPACE) return rc2;  // too large for the workspace: stays flagged
    }
    return BRI_OK;
  }
  if (batch_mergeable(o) && mixed_precision(o->precision)) {
    MixedBatch mb;
    try {
      mb = make_mixed_batch(count, n, k, j, o, true);
    } catch (const std::exception&) {
      return BRI_ERR_UNSUPPORTED;
    }
    if (!o->workspace || o->workspace_bytes < mb.total) return BRI_ERR_WORKSPACE;
    return run_mixed_batch(mb, count, M, n, ldm, i, j, out, ldo, o);
  }
  if (batch_mergeable(o)) {
    BatchPlan bp;
    try {
      bp = make_batch_plan(count, n, k, i, j, elem_size(o->precision), o->reuse);
    } catch (const std::exception&) {
      return BRI_ERR_UNSUPPORTED;
    }
    if (!o->workspace || o->workspace_bytes < bp.total) return BRI_ERR_WORKSPACE;
    return o->precision == BRI_F64 ? run_batch<double>(bp, M, n, ldm, out, ldo, count, o)
                                   : run_batch<float>(bp, M, n, ldm, out, ldo, count, o);
  }
  for (int t = 0; t < count; ++t) {
    bri_opts ot = *o;
    ot.d_info = o->d_info ? o->d_info + t : nullptr;
    const int rc = invert_block(M[t], n[t], ldm[t], k[t], i[t], j[t], out[t], ldo[t], &ot);
    if (rc != BRI_OK) return rc;
  }
  return BRI_OK;
}

size_t bri_blocks_workspace_size(int64_t n, int k, int count, const int* i, const int* j, const bri_opts* o) {
  if (count <= 0 || !i || !j || !o) return 0;
  std::vector<int64_t> nn(count, n);
  std::vector<int> kk(count, k);
  return bri_batched_workspace_size(count, nn.data(), kk.data(), i, j, o);
}

int invert_blocks(const void* M, int64_t n, int64_t ldm, int k, int count, const int* i, const int* j,
                  void* const* out, const int64_t* ldo, const bri_opts* o) {
  if (!M) return -1;
  if (count < 0) return -5;
  if (!i) return -6;
  if (!j) return -7;
  if (!out) return -8;
  if (!ldo) return -9;
  if (!o) return -10;
  if (count == 0) return BRI_OK;
  for (int t = 0; t < count; ++t) {
    const int rc = check_block_args(n, ldm, k, i[t], j[t], ldo[t]);
    if (rc == -5 || rc == -6) return rc - 1;  // i, j are arguments 6 and 7 here
    if (rc == -8) return -9;
    if (rc) return rc;
    if (!out[t]) return -8;
  }
  std::vector<const void*> mm(count, M);
  std::vector<int64_t> nn(count, n), ll(count, ldm);
  std::vector<int> kk(count, k);
  return invert_block_batched(count, mm.data(), nn.data(), ll.data(), kk.data(), i, j, out, ldo, o);
}

}  // extern "C"

// The RbfSource of a matrix-free call sits in the workspace, past the
// status word (the first kAlign bytes of the info region hold both).
constexpr size_t kRbfOffset = 64;
static_assert(kRbfOffset + sizeof(RbfSource) <= kAlign, "RbfSource in the status block");

static size_t rbf_size_of(int64_t m, int k, int i, int j, const bri_opts* o) {
  try {
    return get_plan(3, m, k, i, j, resolve_width(m, k, o), elem_size(o->precision), 0)->layout.total;
  } catch (const std::exception&) {
    return 0;
  }
}

static int check_rbf_args(int64_t npts, int64_t ldx, int d, double sigma, double gamma, int k, int i, int j,
                          int64_t ldo, const bri_opts* o) {
  if (npts < 1) return -2;
  if (d < 1 || ldx < d) return -3;
  if (!(sigma > 0.0)) return -5;
  if (!(gamma > 0.0)) return -6;
  const int64_t m = npts + 1;
  const int rc = check_block_args(m, m, k, i, j, ldo);
  if (rc == -4) return -7;
  if (rc == -5) return -8;
  if (rc == -6) return -9;
  if (rc == -8) return -11;
  if (rc) return rc;
  if (!o) return -12;
  if (!plain_precision(o->precision)) return BRI_ERR_UNSUPPORTED;
  return 0;
}

static int invert_block_rbf_impl(const void* X, int64_t npts, int64_t ldx, int d, double sigma, double gamma, int k,
                                 int i, int j, void* out, int64_t ldo, const bri_opts* o) {
  const int64_t m = npts + 1;
  if (o->pivoting == BRI_PIVOT_AUTO) {
    bri_opts t = *o;
    t.pivoting = BRI_PIVOT_TILE;
    if (!t.d_info) {
      const size_t need = rbf_size_of(m, k, i, j, o);
      if (need == 0 || !o->workspace || o->workspace_bytes < need) return BRI_ERR_WORKSPACE;
      auto cp = get_plan(3, m, k, i, j, resolve_width(m, k, o), elem_size(o->precision), 0);
      t.d_info = reinterpret_cast<int32_t*>(static_cast<char*>(o->workspace) + cp->layout.info_off);
    }
    int rc2 = invert_block_rbf_impl(X, npts, ldx, d, sigma, gamma, k, i, j, out, ldo, &t);
    int32_t h = 0;
    if (rc2 == BRI_OK) rc2 = read_info1(t.d_info, h, o->stream);
    if (rc2 != BRI_OK || h <= 0) return rc2;
    t.pivoting = BRI_PIVOT_PANEL;
    return invert_block_rbf_impl(X, npts, ldx, d, sigma, gamma, k, i, j, out, ldo, &t);
  }
  const int elem = elem_size(o->precision);
  std::shared_ptr<CachedPlan> cp;
  try {
    cp = get_plan(3, m, k, i, j, resolve_width(m, k, o), elem, 0);
  } catch (const std::exception&) {
    return BRI_ERR_UNSUPPORTED;
  }
  if (!o->workspace || o->workspace_bytes < cp->layout.total) return BRI_ERR_WORKSPACE;
  char* ws = static_cast<char*>(o->workspace);
  RbfSource src;
  src.X = X;
  src.ldx = ldx;
  src.npts = static_cast<int32_t>(npts);
  src.d = d;
  src.inv_two_sigma2 = 1.0 / (2.0 * sigma * sigma);
  src.inv_gamma = 1.0 / gamma;
  RbfSource* dsrc = reinterpret_cast<RbfSource*>(ws + cp->layout.info_off + kRbfOffset);
  if (launch_store_rbf(dsrc, src, o->stream) != hipSuccess) return BRI_ERR_HIP;
  Ctx c;
  c.pivoting = o->pivoting;
  c.lu = o->factorization;
  c.M = static_cast<const char*>(X);
  c.n = m;
  c.ldm = m;
  c.b = cp->plan.b;
  c.elem = elem;
  c.rbf = dsrc;
  c.ws = ws;
  c.out = static_cast<char*>(out);
  c.ldo = ldo;
  c.info = o->d_info ? o->d_info : reinterpret_cast<int32_t*>(ws + cp->layout.info_off);
  return execute(*cp, c, o->stream, true);
}

extern "C" {

size_t bri_rbf_workspace_size(int64_t npts, int d, int k, int i, int j, const bri_opts* o) {
  if (!o || o->order != BRI_ORDER_PRINCIPAL || check_rbf_args(npts, d, d, 1.0, 1.0, k, i, j, (npts + k) / k, o) != 0) return 0;
  const int64_t m = npts + 1;
  bool fits;
  const bri_opts ob = with_budget(o, m, k, [&](const bri_opts& r) { return rbf_size_of(m, k, i, j, &r); }, fits);
  return fits ? rbf_size_of(m, k, i, j, &ob) : 0;
}

int invert_block_rbf(const void* X, int64_t npts, int64_t ldx, int d, double sigma, double gamma, int k, int i,
                     int j, void* out, int64_t ldo, const bri_opts* o) {
  if (!X) return -1;
  if (!out) return -10;
  const int rc = check_rbf_args(npts, ldx, d, sigma, gamma, k, i, j, ldo, o);
  if (rc) return rc;
  if (o->order != BRI_ORDER_PRINCIPAL) return BRI_ERR_UNSUPPORTED;
  const int64_t m = npts + 1;
  bool fits;
  const bri_opts ob = with_budget(o, m, k, [&](const bri_opts& r) { return rbf_size_of(m, k, i, j, &r); }, fits);
  if (!fits) return BRI_ERR_WORKSPACE;
  return invert_block_rbf_impl(X, npts, ldx, d, sigma, gamma, k, i, j, out, ldo, &ob);
}

size_t bri_gemm_workspace_size(int count) {
  return count <= 0 ? 0 : align_up(static_cast<size_t>(count) * sizeof(GemmItem)) + kAlign;
}

int bri_gemm(int count, int64_t m, int64_t n, int64_t kk, double alpha, const void* const* A, int64_t lda,
             const void* const* B, int64_t ldb, double beta, void* const* C, int64_t ldc, const bri_opts* o) {
  if (count < 0) return -1;
  if (m < 0 || m > INT_MAX) return -2;
  if (n < 0 || n > INT_MAX) return -3;
  if (kk < 0 || kk > INT_MAX) return -4;
  if (!A && count) return -6;
  if (lda < std::max<int64_t>(1, kk)) return -7;
  if (!B && count) return -8;
  if (ldb < std::max<int64_t>(1, n)) return -9;
  if (!C && count) return -11;
  if (ldc < std::max<int64_t>(1, n)) return -12;
  if (!o) return -13;
  if (!plain_precision(o->precision) && !mixed_precision(o->precision)) return BRI_ERR_UNSUPPORTED;
  if (count == 0 || m == 0 || n == 0) return BRI_OK;
  const size_t need = bri_gemm_workspace_size(count);
  if (!o->workspace || o->workspace_bytes < need) return BRI_ERR_WORKSPACE;
  std::vector<GemmItem> items(count);
  for (int t = 0; t < count; ++t) {
    GemmItem& g = items[t];
    std::memset(&g, 0, sizeof(g));
    g.A = g.B = g.Cin = g.Sub = zero_view();
    g.A.p = A[t];
    g.A.ld = lda;
    g.A.rows = static_cast<int32_t>(m);
    g.A.cols = static_cast<int32_t>(kk);
    g.B.p = B[t];
    g.B.ld = ldb;
    g.B.rows = static_cast<int32_t>(kk);
    g.B.cols = static_cast<int32_t>(n);
    g.Cin = g.A;
    g.Cin.p = C[t];
    g.Cin.ld = ldc;
    g.Cin.rows = static_cast<int32_t>(m);
    g.Cin.cols = static_cast<int32_t>(n);
    g.has_cin = beta != 0.0 ? 1 : 0;
    g.out = C[t];
    g.ldo = ldc;
    g.M = static_cast<int32_t>(m);
    g.N = static_cast<int32_t>(n);
    g.K = static_cast<int32_t>(kk);
    g.alpha = alpha;
    g.beta = beta;
  }
  static std::mutex mu;
  static void* host = nullptr;
  static size_t host_bytes = 0;
  static hipEvent_t ev = nullptr;
  std::lock_guard<std::mutex> lk(mu);
  const size_t bytes = items.size() * sizeof(GemmItem);
  if (ev && hipEventSynchronize(ev) != hipSuccess) return BRI_ERR_HIP;
  if (host_bytes < bytes) {
    if (host) (void)hipHostFree(host);
    host = nullptr;
    if (hipHostMalloc(&host, bytes) != hipSuccess) return BRI_ERR_HIP;
    host_bytes = bytes;
  }
  if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return BRI_ERR_HIP;
  std::memcpy(host, items.data(), bytes);
  if (hipMemcpyAsync(o->workspace, host, bytes, hipMemcpyHostToDevice, o->stream) != hipSuccess) return BRI_ERR_HIP;
  if (hipEventRecord(ev, o->stream) != hipSuccess) return BRI_ERR_HIP;
  GemmLaunch L{};
  L.mode = GEMM_EXPLICIT;
  L.elem = o->precision == BRI_F64 ? 8 : 4;
  L.lp = lp_of(o->precision);
  L.items = o->workspace;
  L.count = count;
  L.w = count;  // plain dense operands: all items take the fast instance
  if (L.lp >= 1) {
    // Split products: the vectorised or split-once instances when every
    // item qualifies, and workspace beyond the descriptors as split scratch.
    bool vec = true;
    for (const GemmItem& g : items) vec = vec && gemm_item_is_lp_vec(g);
    L.ndl = vec ? count : 0;
    L.max_k = static_cast<int32_t>(kk);
    if (vec && o->workspace_bytes > need) {
      L.split = static_cast<char*>(o->workspace) + need;
      L.split_bytes = static_cast<int64_t>(o->workspace_bytes - need);
    }
  }
  const hipError_t e = L.elem == 8 ? launch_gemm<double>(L, static_cast<int>(m), static_cast<int>(n), o->stream)
                                   : launch_gemm<float>(L, static_cast<int>(m), static_cast<int>(n), o->stream);
  return e == hipSuccess ? BRI_OK : BRI_ERR_HIP;
}

static size_t backward_size_of(int64_t n, int k, int i, int j, const bri_opts* o);

static bri_opts backward_budget(const bri_opts* o, int64_t n, int k, int i, int j, bool& fits) {
  return with_budget(o, n, k, [&](const bri_opts& r) { return backward_size_of(n, k, i, j, &r); }, fits);
}

size_t bri_backward_workspace_size(int64_t n, int k, int i, int j, const bri_opts* o) {
  if (!o || check_block_args(n, n, k, i, j, (n + k - 1) / k) != 0) return 0;
  if (!plain_precision(o->precision) || o->order != BRI_ORDER_PRINCIPAL) return 0;
  bool fits;
  const bri_opts ob = backward_budget(o, n, k, i, j, fits);
  return fits ? backward_size_of(n, k, i, j, &ob) : 0;
}

static size_t backward_size_of(int64_t n, int k, int i, int j, const bri_opts* o) {
  const int elem = elem_size(o->precision);
  const int64_t b = (n + k - 1) / k;
  const size_t colbuf = align_up(static_cast<size_t>(k * b) * b * elem);
  const int w = resolve_width(n, k, o);
  size_t plan_ws = 0;
  try {
    plan_ws = std::max(get_plan(1, n, k, 0, i, w, elem, 1)->layout.total, get_plan(1, n, k, 0, j, w, elem, 0)->layout.total);
  } catch (const std::exception&) {
    return 0;
  }
  return 3 * colbuf + align_up(2 * sizeof(GemmItem)) + plan_ws;
}

int invert_block_backward(const void* M, int64_t n, int64_t ldm, int k, int i, int j, const void* G, int64_t ldg,
                          void* grad_M, int64_t ldgm, const bri_opts* o) {
  if (!M) return -1;
  if (!G) return -7;
  if (!grad_M) return -9;
  if (!o) return -11;
  if (o->order != BRI_ORDER_PRINCIPAL) return BRI_ERR_UNSUPPORTED;
  if (n < 1) return -2;
  if (ldm < n) return -3;
  if (k < 2 || k > n) return -4;
  if (i < 0 || i >= k) return -5;
  if (j < 0 || j >= k) return -6;
  const int64_t b = (n + k - 1) / k;
  if (ldg < b) return -8;
  if (ldgm < n) return -10;
  if (b > BRI_MAX_BLOCK) return BRI_ERR_UNSUPPORTED;
  if (!plain_precision(o->precision)) return BRI_ERR_UNSUPPORTED;
  bool fits;
  const bri_opts ob = backward_budget(o, n, k, i, j, fits);
  if (!fits) return BRI_ERR_WORKSPACE;
  o = &ob;
  const size_t need = backward_size_of(n, k, i, j, o);
  if (need == 0) return BRI_ERR_UNSUPPORTED;
  if (!o->workspace || o->workspace_bytes < need) return BRI_ERR_WORKSPACE;
  const int elem = elem_size(o->precision);
  const size_t colbuf = align_up(static_cast<size_t>(k * b) * b * elem);
  char* ws = static_cast<char*>(o->workspace);
  char* U = ws;                // block column i of (M^T)^{-1} = (N_{i,:})^T
  char* V = ws + colbuf;       // block column j of M^{-1}    = N_{:,j}
  char* T1 = ws + 2 * colbuf;  // U G
  char* desc = ws + 3 * colbuf;
  char* rest = desc + align_up(2 * sizeof(GemmItem));
  bri_opts oc = *o;
  oc.workspace = rest;
  oc.workspace_bytes = o->workspace_bytes - (rest - ws);
  int rc = bri_block_column(M, n, ldm, k, i, 1, U, b, &oc);
  if (rc != BRI_OK) return rc;
  rc = bri_block_column(M, n, ldm, k, j, 0, V, b, &oc);
  if (rc != BRI_OK) return rc;
  // T1 = U G (kb x b), grad_M = -T1 V^T restricted to n x n.
  GemmItem g[2];
  std::memset(g, 0, sizeof(g));
  for (int t = 0; t < 2; ++t) g[t].A = g[t].B = g[t].Cin = g[t].Sub = zero_view();
  g[0].A.p = U;
  g[0].A.ld = b;
  g[0].A.rows = static_cast<int32_t>(k * b);
  g[0].A.cols = static_cast<int32_t>(b);
  g[0].B.p = G;
  g[0].B.ld = ldg;
  g[0].B.rows = static_cast<int32_t>(b);
  g[0].B.cols = static_cast<int32_t>(b);
  g[0].out = T1;
  g[0].ldo = b;
  g[0].M = static_cast<int32_t>(n);
  g[0].N = static_cast<int32_t>(b);
  g[0].K = static_cast<int32_t>(b);
  g[0].alpha = 1.0;
  g[1].A.p = T1;
  g[1].A.ld = b;
  g[1].A.rows = static_cast<int32_t>(n);
  g[1].A.cols = static_cast<int32_t>(b);
  g[1].B.p = V;  // element (t, c) of V^T is V[c][t]
  g[1].B.ld = b;
  g[1].B.trans = 1;
  g[1].B.rows = static_cast<int32_t>(b);
  g[1].B.cols = static_cast<int32_t>(n);
  g[1].out = grad_M;
  g[1].ldo = ldgm;
  g[1].M = static_cast<int32_t>(n);
  g[1].N = static_cast<int32_t>(n);
  g[1].K = static_cast<int32_t>(b);
  g[1].alpha = -1.0;
  static std::mutex mu;
  static void* host = nullptr;
  static hipEvent_t ev = nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (!host) {
    if (hipHostMalloc(&host, 2 * sizeof(GemmItem)) != hipSuccess) return BRI_ERR_HIP;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return BRI_ERR_HIP;
  } else if (hipEventSynchronize(ev) != hipSuccess) {
    return BRI_ERR_HIP;
  }
  std::memcpy(host, g, sizeof(g));
  if (hipMemcpyAsync(desc, host, sizeof(g), hipMemcpyHostToDevice, o->stream) != hipSuccess) return BRI_ERR_HIP;
  if (hipEventRecord(ev, o->stream) != hipSuccess) return BRI_ERR_HIP;
  GemmLaunch L{};
  L.mode = GEMM_EXPLICIT;
  L.elem = elem;
  L.count = 1;
  L.w = 1;  // stored dense operands (U, G, T1, V^T)
  L.items = desc;
  hipError_t e = elem == 8 ? launch_gemm<double>(L, static_cast<int>(n), static_cast<int>(b), o->stream)
                           : launch_gemm<float>(L, static_cast<int>(n), static_cast<int>(b), o->stream);
  if (e != hipSuccess) return BRI_ERR_HIP;
  L.items = desc + sizeof(GemmItem);
  e = elem == 8 ? launch_gemm<double>(L, static_cast<int>(n), static_cast<int>(n), o->stream)
                : launch_gemm<float>(L, static_cast<int>(n), static_cast<int>(n), o->stream);
  return e == hipSuccess ? BRI_OK : BRI_ERR_HIP;
}

}  // extern "C"
