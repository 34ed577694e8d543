// Autotuner: which LU variant a factorisation launch takes and which tile
// shape the FP64 explicit products take, measured on this GPU by
// bri_autotune() and kept in a text cache file that later processes load.
//
// Cache file (one decision per line; '#' starts a comment):
//   lu <count> <b> <kind>                      kind: 0 tile steps, 2 recursive
//   product <elem> <tri> <count> <m> <n> <shape>
// Counts and orders are bucketed to the power of two at or below them, and a
// lookup takes the entry of its bucket.  Without a cache (or an entry) the
// built-in rules apply.  The file is $BRI_TUNE_CACHE, else
// $HOME/.cache/bri-mi355x/tune.txt.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <sys/stat.h>
#include <tuple>
#include <vector>

#include "../../include/bri.h"
#include "bri_internal.h"
#include "bri_kernels.h"

namespace bri {

thread_local int g_force_shape = -1;
thread_local int g_force_lu = -1;

namespace {

int bucket(int64_t x) {
  int p = 0;
  while ((int64_t(2) << p) <= x) ++p;
  return x <= 0 ? -1 : p;
}

struct TuneTable {
  std::mutex mu;
  bool loaded = false;
  std::map<std::pair<int, int>, int> lu;                                // (count bucket, b bucket) -> kind
  std::map<std::tuple<int, int, int, int, int>, int> product;           // (elem, tri, count, m, n buckets) -> shape
};
TuneTable& table() {
  static TuneTable t;
  return t;
}

std::string default_path() {
  if (const char* p = std::getenv("BRI_TUNE_CACHE")) return p;
  const char* home = std::getenv("HOME");
  return std::string(home ? home : ".") + "/.cache/bri-mi355x/tune.txt";
}

// Parses a cache file into t (entries replace those of their bucket).
// Returns the entries read, or -1 when the file cannot be opened.
int load_file(TuneTable& t, const std::string& path) {
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return -1;
  char line[256];
  int n = 0;
  while (std::fgets(line, sizeof(line), f)) {
    char* hash = std::strchr(line, '#');
    if (hash) *hash = 0;
    char kind[32];
    long a = 0, b = 0, c = 0, d = 0, e = 0, g = 0;
    if (std::sscanf(line, "%31s", kind) != 1) continue;
    if (!std::strcmp(kind, "lu") && std::sscanf(line, "%*s %ld %ld %ld", &a, &b, &c) == 3) {
      t.lu[{bucket(a), bucket(b)}] = static_cast<int>(c);
      ++n;
    } else if (!std::strcmp(kind, "product") &&
               std::sscanf(line, "%*s %ld %ld %ld %ld %ld %ld", &a, &b, &c, &d, &e, &g) == 6) {
      t.product[std::make_tuple(static_cast<int>(a), static_cast<int>(b), bucket(c), bucket(d), bucket(e))] =
          static_cast<int>(g);
      ++n;
    }
  }
  std::fclose(f);
  return n;
}

TuneTable& loaded_table() {
  TuneTable& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  if (!t.loaded) {
    t.loaded = true;
    (void)load_file(t, default_path());
  }
  return t;
}

void make_dirs(const std::string& path) {
  for (size_t p = path.find('/', 1); p != std::string::npos; p = path.find('/', p + 1))
    (void)mkdir(path.substr(0, p).c_str(), 0755);
}

}  // namespace

int tuned_lu_kind(int count, int b) {
  TuneTable& t = loaded_table();
  std::lock_guard<std::mutex> g(t.mu);
  auto it = t.lu.find({bucket(count), bucket(b)});
  return it == t.lu.end() ? -1 : it->second;
}

int tuned_product_shape(int elem, int tri, int count, int m, int n) {
  TuneTable& t = loaded_table();
  std::lock_guard<std::mutex> g(t.mu);
  auto it = t.product.find(std::make_tuple(elem, tri ? 1 : 0, bucket(count), bucket(m), bucket(n)));
  return it == t.product.end() ? -1 : it->second;
}

namespace {

// Mean milliseconds of reps runs of fn (one untimed run first); prep runs
// before every run, outside the timed part.
template <typename F, typename P>
double time_ms(hipStream_t st, int reps, F fn, P prep) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.0;
  double total = 0.0;
  bool ok = true;
  for (int r = -1; r < reps && ok; ++r) {
    prep();
    ok = hipEventRecord(a, st) == hipSuccess && fn() == hipSuccess && hipEventRecord(b, st) == hipSuccess &&
         hipEventSynchronize(b) == hipSuccess;
    float ms = 0.f;
    if (ok && r >= 0 && hipEventElapsedTime(&ms, a, b) == hipSuccess) total += ms;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ok ? total / reps : -1.0;
}

DView plain_view(void* p, int64_t ld, int rows, int cols, int tri) {
  DView v;
  std::memset(&v, 0, sizeof(v));
  v.p = p;
  v.ld = ld;
  v.rows = rows;
  v.cols = cols;
  v.diag = -(1 << 30);
  v.tri = static_cast<int16_t>(tri);
  return v;
}

}  // namespace
}  // namespace bri

using namespace bri;

extern "C" {

int bri_tune_load(const char* path) {
  TuneTable& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  t.loaded = true;
  t.lu.clear();
  t.product.clear();
  const int n = load_file(t, path ? std::string(path) : default_path());
  return n < 0 ? BRI_ERR_UNSUPPORTED : n;
}

int bri_autotune(const bri_opts* o, const char* path) {
  if (!o) return -1;
  if (!o->workspace || o->workspace_bytes < (size_t(64) << 20)) return BRI_ERR_WORKSPACE;
  hipStream_t st = o->stream;
  char* ws = static_cast<char*>(o->workspace);
  const size_t cap = o->workspace_bytes;
  std::vector<std::string> lines;
  const size_t kAl = 256;
  auto al = [&](size_t x) { return (x + kAl - 1) / kAl * kAl; };
  // ---- FP64 explicit products: C = C - A B on count items of order s -------
  for (int tri = 0; tri <= 1; ++tri) {
    for (int count : {1, 4, 16, 64}) {
      for (int s : {256, 512, 1024, 2048}) {
        const size_t mat = al(size_t(s) * s * 8);
        const size_t need = 3 * mat * count + al(sizeof(GemmItem) * count);
        if (need > cap) continue;
        std::vector<GemmItem> items(count);
        for (int t = 0; t < count; ++t) {
          char* base = ws + 3 * mat * t;
          GemmItem& g = items[t];
          std::memset(&g, 0, sizeof(g));
          g.A = plain_view(base, s, s, s, tri);
          g.B = plain_view(base + mat, s, s, s, 0);
          g.Cin = plain_view(base + 2 * mat, s, s, s, 0);
          g.Sub = plain_view(nullptr, 0, 0, 0, 0);
          g.has_cin = 1;
          g.out = base + 2 * mat;
          g.ldo = s;
          g.M = g.N = g.K = s;
          g.alpha = -1.0;
          g.beta = 1.0;
        }
        char* desc = ws + 3 * mat * count;
        if (hipMemcpy(desc, items.data(), sizeof(GemmItem) * count, hipMemcpyHostToDevice) != hipSuccess)
          return BRI_ERR_HIP;
        if (hipMemsetAsync(ws, 0, 3 * mat * count, st) != hipSuccess) return BRI_ERR_HIP;
        GemmLaunch L{};
        L.mode = GEMM_EXPLICIT;
        L.elem = 8;
        L.items = desc;
        L.count = count;
        L.w = count;
        L.ndl = count;
        L.tri = tri;
        int best = -1;
        double best_ms = 0.0;
        for (int shape : {kShapeDl128, kShapeDl64, kShapeDl256, kShapeDl128w}) {
          g_force_shape = shape;
          const double ms = time_ms(st, 3, [&] { return launch_gemm<double>(L, s, s, st); }, [] {});
          g_force_shape = -1;
          if (ms > 0 && (best < 0 || ms < best_ms)) {
            best = shape;
            best_ms = ms;
          }
        }
        if (best >= 0)
          lines.push_back("product 8 " + std::to_string(tri) + " " + std::to_string(count) + " " +
                          std::to_string(s) + " " + std::to_string(s) + " " + std::to_string(best) + "  # " +
                          std::to_string(best_ms) + " ms");
      }
    }
  }
  // ---- LU variant of a factorisation launch of count matrices of order b ---
  for (int count : {1, 4, 16, 64}) {
    for (int b : {256, 512, 1024, 2048}) {
      const size_t mat = al(size_t(b) * b * 8);
      const size_t per = 2 * mat + al(size_t(b) * 4) + al(sizeof(int32_t) * kSwapWords) + al(kAuxElems * 8);
      const size_t need = per * count + al(sizeof(LuItem) * count) + kAl;
      if (need > cap) continue;
      std::vector<LuItem> items(count);
      int32_t* info = reinterpret_cast<int32_t*>(ws + per * count + al(sizeof(LuItem) * count));
      for (int t = 0; t < count; ++t) {
        char* base = ws + per * t;
        LuItem& it = items[t];
        std::memset(&it, 0, sizeof(it));
        it.a = base;
        it.tmp = base + mat;
        it.perm = reinterpret_cast<int32_t*>(base + 2 * mat);
        it.swaps = reinterpret_cast<int32_t*>(base + 2 * mat + al(size_t(b) * 4));
        it.aux = base + 2 * mat + al(size_t(b) * 4) + al(sizeof(int32_t) * kSwapWords);
        it.info = info;
        it.b = b;
      }
      LuItem* d_items = reinterpret_cast<LuItem*>(ws + per * count);
      if (hipMemcpy(d_items, items.data(), sizeof(LuItem) * count, hipMemcpyHostToDevice) != hipSuccess)
        return BRI_ERR_HIP;
      auto prep = [&] { (void)launch_fill_diag_dominant(d_items, count, b, st); };
      const double t_tile = time_ms(st, 2, [&] {
        hipError_t e = launch_getrf_tile<double>(d_items, count, b, false, st);
        return e == hipSuccess ? launch_trtri<double>(d_items, count, b, true, st) : e;
      }, prep);
      const double t_rec = getrf_rec_possible(b)
                               ? time_ms(st, 2, [&] { return launch_getrf_rec<double>(d_items, count, b, false, 0, nullptr, st); },
                                         prep)
                               : -1.0;
      if (t_tile > 0 && t_rec > 0)
        lines.push_back("lu " + std::to_string(count) + " " + std::to_string(b) + " " +
                        std::to_string(t_rec < t_tile ? LU_RECURSIVE : LU_TILE) + "  # tile " +
                        std::to_string(t_tile) + " ms, recursive " + std::to_string(t_rec) + " ms");
    }
  }
  // ---- keep the decisions and write the cache -------------------------------
  const std::string file = path ? std::string(path) : default_path();
  make_dirs(file);
  FILE* f = std::fopen(file.c_str(), "w");
  if (!f) return BRI_ERR_UNSUPPORTED;
  std::fprintf(f, "# bri-mi355x tuning cache (bri_autotune)\n");
  for (const std::string& l : lines) std::fprintf(f, "%s\n", l.c_str());
  std::fclose(f);
  const int n = bri_tune_load(file.c_str());
  return n < 0 ? n : static_cast<int>(lines.size());
}

}  // extern "C"
