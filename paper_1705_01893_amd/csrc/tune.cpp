// Transform layouts of the real chunk transforms and their plan-time autotuner.
//
// A chunk of n = 2M real samples is transformed as M complex values with the four-step
// split M = M1 * M2: column transforms of length M2 (pass A forward, pass C inverse; a column
// item holds cb adjacent columns) and row transforms of length M1 (pass B, two rows per item).
// Several splits, column-block widths and radix orders fit the passes' tiles; the tuner times
// each candidate on copies of the chunk length and keeps the fastest.
#include <hip/hip_runtime.h>

#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "plan.h"

// identifies the library build in the persisted tuner choices (the build script passes a hash
// of the sources)
#ifndef MM_BUILD_ID
#define MM_BUILD_ID "unversioned"
#endif

namespace mm {

namespace {

int64_t pow2floor(int64_t x) {
  while (x & (x - 1)) x &= x - 1;
  return x;
}

// Radix schedule for a 5-smooth length: the fewest stages over the radices the precision's
// register budget allows (radix_ok), ties broken toward the smaller largest radix, then the
// larger smallest one; ascending order, or descending with largest_first.
std::vector<int8_t> radices(int64_t L, bool largest_first, bool f64) {
  int e[3] = {0, 0, 0};
  const int pr[3] = {2, 3, 5};
  for (int i = 0; i < 3; ++i)
    while (L % pr[i] == 0) {
      L /= pr[i];
      ++e[i];
    }
  std::vector<int> rs;
  for (int R = 2; R <= 25; ++R)
    if (radix_ok(R, f64)) rs.push_back(R);
  const int nr = (int)rs.size();
  // best[a][b][c] = (stages, the radices) for 2^a 3^b 5^c, by increasing exponents
  const int A = e[0] + 1, B = e[1] + 1, C = e[2] + 1;
  std::vector<int> cnt(A * B * C, 1 << 20), last(A * B * C, 0), peak(A * B * C, 0), low(A * B * C, 1 << 20);
  cnt[0] = 0;
  for (int a = 0; a < A; ++a)
    for (int b = 0; b < B; ++b)
      for (int c = 0; c < C; ++c) {
        const int id = (a * B + b) * C + c;
        if (id == 0) continue;
        for (int k = 0; k < nr; ++k) {
          int r = rs[k], x = 0, y = 0, z = 0;
          while (r % 2 == 0) r /= 2, ++x;
          while (r % 3 == 0) r /= 3, ++y;
          while (r % 5 == 0) r /= 5, ++z;
          if (x > a || y > b || z > c) continue;
          const int prev = ((a - x) * B + (b - y)) * C + (c - z);
          if (cnt[prev] >= (1 << 20)) continue;
          const int n = cnt[prev] + 1, pk = std::max(peak[prev], rs[k]), lo = std::min(low[prev], rs[k]);
          if (n < cnt[id] || (n == cnt[id] && (pk < peak[id] || (pk == peak[id] && lo > low[id])))) {
            cnt[id] = n;
            last[id] = rs[k];
            peak[id] = pk;
            low[id] = lo;
          }
        }
      }
  std::vector<int8_t> r;
  for (int a = e[0], b = e[1], c = e[2]; a + b + c > 0;) {
    const int id = (a * B + b) * C + c;
    int q = last[id];
    r.push_back((int8_t)q);
    while (q % 2 == 0) q /= 2, --a;
    while (q % 3 == 0) q /= 3, --b;
    while (q % 5 == 0) q /= 5, --c;
  }
  std::sort(r.begin(), r.end());
  if (largest_first) std::reverse(r.begin(), r.end());
  return r;
}

void omega_table(int64_t L, int64_t count, int64_t stride, std::vector<double2>& out) {
  // out += exp(-2 pi i (q * stride) / L), q < count
  for (int64_t q = 0; q < count; ++q) {
    const int64_t e = (q * stride) % L;
    const double a = -2.0 * M_PI * (double)e / (double)L;
    out.push_back(make_double2(std::cos(a), std::sin(a)));
  }
}

}  // namespace

int tile_cap_ac(bool f64) { return kBlock * (f64 ? Ept<double>::v : Ept<float>::v); }

int tile_cap_b(bool f64) {
  // a row item (two rows) holds at most Ept elements per thread of the row pass, and its tile
  // plus the chi^2 reduction slots fit 64 KB of LDS
  const size_t csz = f64 ? sizeof(double2) : sizeof(float2);
  return std::min<int>(kBlockB * (f64 ? Ept<double>::v : Ept<float>::v),
                       (int)((65536 - (kBlockB / 64) * sizeof(double)) / csz));
}

std::vector<Layout> layout_candidates(int64_t M, bool f64) {
  const int cap = tile_cap_ac(f64), row_cap = tile_cap_b(f64);
  const int bmax = f64 ? 8 : 16;  // 128-byte rows of column blocks
  struct Scored {
    double score;
    Layout L;
  };
  std::vector<Scored> v;
  for (int64_t m2 = 1; m2 <= M && m2 <= cap; ++m2) {
    if (M % m2) continue;
    const int64_t m1 = M / m2;
    if (2 * m1 > row_cap) continue;
    const int64_t bfull = pow2floor(std::min<int64_t>(bmax, m1));
    const int64_t b = std::min<int64_t>(bfull, pow2floor(cap / m2));
    if (b < 1) continue;
    // static rule: full column blocks first, then row lengths that keep column runs on 128-byte lines
    // (M1 a multiple of cb), then the split closest to sqrt(M)
    const double score = std::fabs(std::log((double)m2) - 0.5 * std::log((double)M)) + (b < bfull ? 4.0 : 0.0) +
                         (m1 % b != 0 ? 2.0 : 0.0);
    for (int order = 0; order < 2; ++order) {
      Layout L;
      L.M1 = m1;
      L.M2 = m2;
      L.cb = (int)b;
      L.r1 = radices(m1, order == 1, f64);
      L.r2 = radices(m2, order == 1, f64);
      if ((int)L.r1.size() > kMaxStages || (int)L.r2.size() > kMaxStages) continue;
      // the second radix order is a distinct candidate only when it differs
      if (order == 1 && L.r1 == radices(m1, false, f64) && L.r2 == radices(m2, false, f64)) continue;
      v.push_back({score + 1e-3 * order, L});
    }
  }
  std::stable_sort(v.begin(), v.end(), [](const Scored& a, const Scored& b) { return a.score < b.score; });
  std::vector<Layout> out;
  for (auto& s : v) out.push_back(s.L);
  return out;
}

void make_class(int64_t M, const Layout& L, std::vector<double2>& tw, DevClass& k) {
  std::memset(&k, 0, sizeof(k));
  k.M = (int32_t)M;
  k.M1 = (int32_t)L.M1;
  k.M2 = (int32_t)L.M2;
  k.nr1 = (int32_t)L.r1.size();
  k.nr2 = (int32_t)L.r2.size();
  std::copy(L.r1.begin(), L.r1.end(), k.rad1);
  std::copy(L.r2.begin(), L.r2.end(), k.rad2);
  k.tw1 = (int64_t)tw.size();
  omega_table(L.M1, L.M1, 1, tw);
  k.tw2 = (int64_t)tw.size();
  omega_table(L.M2, L.M2, 1, tw);
  const int64_t L2 = 2 * M;
  int lb = 0;
  while ((int64_t(1) << (2 * lb)) < L2) ++lb;  // 2^lb >= sqrt(2M)
  const int64_t lo = int64_t(1) << lb;
  const int64_t nhi = (L2 + lo - 1) / lo;
  k.lb = lb;
  k.twlo = (int64_t)tw.size();
  omega_table(L2, lo, 1, tw);
  k.twhi = (int64_t)tw.size();
  omega_table(L2, nhi, lo, tw);
}

bool row_fuse(int M1, bool f64) { return 4 * M1 <= tile_cap_b(f64); }

void append_col_items(int32_t c, const DevChunk& ch, std::vector<ItemAC>& itemsAC) {
  for (int32_t j1 = 0; j1 < ch.M1; j1 += ch.cb) itemsAC.push_back({c, j1});
}

void append_row_items(int32_t c, const DevChunk& ch, std::vector<ItemB>& itemsB, bool fuse) {
  const int M2 = ch.M2;
  // rows k2 and M2 - k2 pair up (bins k and M - k); row 0 (and row M2/2) pair with themselves
  itemsB.push_back({c, 0, M2 % 2 == 0 ? M2 / 2 : 0, 0});
  const int last = M2 % 2 == 0 ? M2 / 2 - 1 : (M2 - 1) / 2;
  for (int k2 = 1; k2 <= last; ++k2) {
    if (fuse && k2 + 1 <= last) {
      itemsB.push_back({c, k2, M2 - k2, k2 + 1});
      ++k2;
    } else {
      itemsB.push_back({c, k2, M2 - k2, 0});
    }
  }
}

namespace {

std::mutex g_tune_mu;
// (persisted cache file or "", M, precision, streams pass A reads) -> candidate index
std::map<std::tuple<std::string, int64_t, int, int>, int> g_tune_cache;

// Persisted choices.  With the environment variable MM_TUNE_CACHE naming a file, every measured
// choice is also written there, one line per choice: the device architecture, the HIP runtime
// version, the library build, the chunk half-length M, the precision and the candidate count,
// then the chosen index.  A process with the same device, runtime and build reads the choice
// back instead of timing the candidates again.  Lines of other keys are kept; lines that do not
// parse are dropped when the file is next written (a temporary file renamed over it).
std::string persisted_key(int64_t M, bool f64, int a_streams, int ncand) {
  int dev = 0, rt = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
  if (hipRuntimeGetVersion(&rt) != hipSuccess) rt = 0;
  std::ostringstream k;
  k << prop.gcnArchName << ' ' << rt << ' ' << MM_BUILD_ID << ' ' << M << ' ' << (f64 ? "f64" : "f32") << " a"
    << a_streams << ' ' << ncand;
  return k.str();
}

std::map<std::string, int> read_persisted(const std::string& path) {
  std::map<std::string, int> out;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream ls(line);
    std::vector<std::string> tok;
    std::string t;
    while (ls >> t) tok.push_back(t);
    // the key's fields, then the chosen index
    if (tok.size() < 2) continue;
    char* end = nullptr;
    const long v = std::strtol(tok.back().c_str(), &end, 10);
    if (!end || *end || v < 0 || v >= (long)kTuneMaxCandidates) continue;
    std::string k = tok[0];
    for (size_t i = 1; i + 1 < tok.size(); ++i) k += ' ' + tok[i];
    out[k] = (int)v;
  }
  return out;
}

void write_persisted(const std::string& path, const std::string& key, int value) {
  std::map<std::string, int> all = read_persisted(path);
  all[key] = value;
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  {
    std::ofstream o(tmp, std::ios::trunc);
    if (!o) return;
    for (const auto& kv : all) o << kv.first << ' ' << kv.second << '\n';
    if (!o) return;
  }
  if (std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}

// Passes A-C (filter on) over K copies of a length-2M chunk under one layout: the device
// tables and work lists (carved from the tuner's scratch), kept for repeated timing.
struct LayoutRun {
  std::vector<double2> tw;
  std::vector<float2> tw32;
  std::vector<DevClass> cls;
  std::vector<DevChunk> chunks;
  std::vector<ItemAC> itemsAC;
  std::vector<ItemB> itemsB;
  DevPlan P;
  const ItemAC* dac = nullptr;
  const ItemB* db = nullptr;
  int nac = 0, nb = 0;
  size_t lds_ac = 0, lds_c = 0, lds_b = 0;

  void tables(int64_t M, bool f64, const Layout& L, int64_t K) {
    cls.resize(1);
    make_class(M, L, tw, cls[0]);
    tw32.resize(tw.size());
    for (size_t i = 0; i < tw.size(); ++i) tw32[i] = make_float2((float)tw[i].x, (float)tw[i].y);
    chunks.resize(K);
    for (int64_t c = 0; c < K; ++c) {
      DevChunk& ch = chunks[c];
      std::memset(&ch, 0, sizeof(ch));
      ch.off = c * 2 * M;
      ch.n = (int32_t)(2 * M);
      ch.M = (int32_t)M;
      ch.M1 = (int32_t)L.M1;
      ch.M2 = (int32_t)L.M2;
      ch.cb = L.cb;
      while ((1 << (ch.lgb + 1)) <= ch.cb) ++ch.lgb;
      ch.df = 1.0 / (double)ch.n;
      ch.sigma2 = 1.0;
      ch.fknee = 0.1;
      ch.alpha = -2.0;
      ch.tau = 1.0;
      ch.inv_tau = 1.0;
      ch.nbar0 = 0.0;
      ch.spec_off = c * (M + 1);
      ch.inv_M = 1.0 / (double)M;
      ch.lg0 = std::log2(ch.df / ch.fknee);
      ch.xoff = c * ((M + kWorkAlign - 1) / kWorkAlign * kWorkAlign);
      append_col_items((int32_t)c, ch, itemsAC);
      append_row_items((int32_t)c, ch, itemsB, row_fuse(L.M1, f64));
    }
  }

  // device bytes of the tables (what prepare carves)
  size_t bytes(int64_t M, bool f64, const Layout& L, int64_t K) {
    tables(M, f64, L, K);
    Arena a;
    a.take(chunks.size() * sizeof(DevChunk));
    a.take(sizeof(DevClass));
    a.take(tw.size() * sizeof(double2));
    a.take(tw32.size() * sizeof(float2));
    a.take(itemsAC.size() * sizeof(ItemAC));
    a.take(itemsB.size() * sizeof(ItemB));
    return a.used;
  }

  bool prepare(int64_t M, bool f64, const Layout& L, int64_t K, const double* spec, Arena& ar, hipStream_t s) {
    tables(M, f64, L, K);
    auto put = [&](const void* src, size_t n, void** dst) {
      *dst = ar.take(n);
      return *dst && (n == 0 || hipMemcpyAsync(*dst, src, n, hipMemcpyHostToDevice, s) == hipSuccess);
    };
    void *pch, *pcl, *ptw, *ptw32, *pac, *pb;
    if (!put(chunks.data(), chunks.size() * sizeof(DevChunk), &pch) || !put(cls.data(), sizeof(DevClass), &pcl) ||
        !put(tw.data(), tw.size() * sizeof(double2), &ptw) || !put(tw32.data(), tw32.size() * sizeof(float2), &ptw32) ||
        !put(itemsAC.data(), itemsAC.size() * sizeof(ItemAC), &pac) ||
        !put(itemsB.data(), itemsB.size() * sizeof(ItemB), &pb))
      return false;
    dac = (const ItemAC*)pac;
    db = (const ItemB*)pb;
    nac = (int)itemsAC.size();
    nb = (int)itemsB.size();
    std::memset(&P, 0, sizeof(P));
    P.precision = f64 ? MM_FP64 : MM_MIXED;
    P.all_pow2 = 1;
    for (int8_t r : L.r1) P.all_pow2 &= (r == 2 || r == 4 || r == 8);
    for (int8_t r : L.r2) P.all_pow2 &= (r == 2 || r == 4 || r == 8);
    P.nsamp = K * 2 * M;
    P.nchunk = (int32_t)K;
    P.chunks = (const DevChunk*)pch;
    P.classes = (const DevClass*)pcl;
    P.tw64 = (const double2*)ptw;
    P.tw32 = (const float2*)ptw32;
    // the power-law values only need to be finite: every candidate reads the same table
    P.spec = spec;
    const size_t csz = f64 ? sizeof(double2) : sizeof(float2);
    const bool wl = !(f64 && P.all_pow2) && wave_cols(L.M2, L.cb, (int)csz);
    P.col_wave = wl ? ((!f64 && L.M2 == 1024 && L.cb == kColWaves) ? 3 : 1) : 0;
    lds_ac = (size_t)col_tile_elems(L.M2, L.cb, (int)csz, false) * csz;
    lds_c = (size_t)col_tile_elems(L.M2, L.cb, (int)csz, wl) * csz;
    lds_b = (size_t)(row_fuse(L.M1, f64) ? 4 : 2) * L.M1 * csz;
    return true;
  }

  // pm: null for a pass A that reads d alone, else P m (and its second half with pmb_off set)
  bool run(void* din, void* dwork, const void* pm, hipStream_t s) const {
    return launch_pass_a(P, dac, nac, din, nullptr, pm ? SRC_D_MINUS_PMBUF : SRC_D, dwork, lds_ac, s, pm) ==
               hipSuccess &&
           launch_pass_b(P, db, nb, dwork, B_FILTER, GAIN_MESSENGER, 1.0, 1.0, nullptr, lds_b, s) == hipSuccess &&
           launch_pass_c(P, dac, nac, dwork, lds_c, s) == hipSuccess;
  }
};

// copies of the chunk timed per launch, and the bytes of one copy in the work buffers
void tune_shape(int64_t M, bool f64, int64_t* K, size_t* buf_bytes) {
  *K = std::max<int64_t>(1, kTuneElements / M);
  const int64_t Mp = (M + kWorkAlign - 1) / kWorkAlign * kWorkAlign;
  *buf_bytes = (size_t)(*K) * Mp * (f64 ? sizeof(double2) : sizeof(float2));
}

}  // namespace

bool tune_wanted(int64_t M, size_t ncand) { return ncand > 1 && M >= kTuneMinM; }

size_t tune_scratch_bytes(int64_t M, bool f64, const std::vector<Layout>& cands, int a_streams) {
  if (!tune_wanted(M, cands.size())) return 0;
  int64_t K;
  size_t bb;
  tune_shape(M, f64, &K, &bb);
  Arena a;
  a.take(bb);
  a.take(bb);
  if (a_streams > 1) a.take((size_t)(a_streams - 1) * bb);
  if (f64) a.take((size_t)K * (M + 1) * sizeof(double));
  const int ncand = (int)std::min<size_t>(cands.size(), kTuneMaxCandidates);
  size_t t = a.used;
  for (int i = 0; i < ncand; ++i) {
    LayoutRun r;
    t = (t + 255) / 256 * 256 + r.bytes(M, f64, cands[i], K);
  }
  return t + 256;
}

int tune_layout(int64_t M, bool f64, const std::vector<Layout>& cands, int a_streams, hipStream_t s, void* scratch,
                size_t scratch_bytes) {
  if (!tune_wanted(M, cands.size())) return 0;
  a_streams = std::min(std::max(a_streams, 1), 3);
  const char* env = std::getenv("MM_TUNE_CACHE");
  const std::string path = env ? env : "";
  const auto key = std::make_tuple(path, M, f64 ? 0 : 1, a_streams);
  const int ncand = (int)std::min<size_t>(cands.size(), kTuneMaxCandidates);
  std::string pkey;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) return it->second;
    if (!path.empty()) {
      pkey = persisted_key(M, f64, a_streams, ncand);
      const std::map<std::string, int> saved = read_persisted(path);
      auto ps = pkey.empty() ? saved.end() : saved.find(pkey);
      if (ps != saved.end() && ps->second < ncand) {
        g_tune_cache[key] = ps->second;
        return ps->second;
      }
    }
  }
  int64_t K;
  size_t bb;
  tune_shape(M, f64, &K, &bb);
  Arena ar;
  ar.base = (char*)scratch;
  ar.cap = scratch_bytes;
  void* din = ar.take(bb);
  void* dwork = ar.take(bb);
  void* pm = a_streams > 1 ? ar.take((size_t)(a_streams - 1) * bb) : nullptr;
  double* spec = nullptr;
  if (f64) spec = (double*)ar.take((size_t)K * (M + 1) * sizeof(double));
  if (!din || !dwork || (a_streams > 1 && !pm) || (f64 && !spec)) return 0;
  int best = 0;
  // every candidate prepared and warmed up, then timed round-robin (best of kTuneReps each), so
  // that clock and cache drift during the plan affects all of them alike
  std::vector<std::unique_ptr<LayoutRun>> runs;
  std::vector<double> t(ncand, -1.0);
  bool ok = launch_fill_i64((int64_t*)din, (int64_t)(bb / sizeof(int64_t)), 0, s) == hipSuccess;
  if (ok && pm)
    ok = launch_fill_i64((int64_t*)pm, (int64_t)((size_t)(a_streams - 1) * bb / sizeof(int64_t)), 0, s) ==
         hipSuccess;
  for (int i = 0; ok && i < ncand; ++i) {
    runs.emplace_back(new LayoutRun);
    ok = runs[i]->prepare(M, f64, cands[i], K, spec, ar, s);
    // a composite plan's P_B m half follows the P_A m half (offsets in complex pairs)
    if (ok && a_streams == 3) runs[i]->P.pmb_off = K * M;
    if (ok && f64 && i == 0) ok = launch_spectrum(runs[0]->P, spec, s) == hipSuccess;
    ok = ok && runs[i]->run(din, dwork, pm, s);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ok = ok && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  for (int rep = 0; ok && rep < kTuneReps; ++rep)
    for (int i = 0; ok && i < ncand; ++i) {
      float ms = 0.f;
      ok = hipEventRecord(e0, s) == hipSuccess && runs[i]->run(din, dwork, pm, s) &&
           hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
           hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
      if (ok && (t[i] < 0 || ms < t[i])) t[i] = ms;
    }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  (void)hipGetLastError();
  if (ok) {
    double tbest = t[0];
    for (int i = 1; i < ncand; ++i)
      if (t[i] < tbest * 0.98) {  // a clear win over the better-ranked layouts
        tbest = t[i];
        best = i;
      }
  }
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune_cache[key] = best;
  if (ok && !pkey.empty()) write_persisted(path, pkey, best);
  return best;
}

}  // namespace mm
