// Plan construction for libmm: validation, transform splits, twiddle tables,
// work lists, and the pixel-tile sort that makes binning deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "mm.h"
#include "plan.h"

namespace mm {

thread_local std::string g_last_error;

mm_status fail(mm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

static bool five_smooth(int64_t x) {
  if (x < 1) return false;
  for (int p : {2, 3, 5})
    while (x % p == 0) x /= p;
  return x == 1;
}

template <typename X>
static mm_status upload(mm_plan_s* pl, const std::vector<X>& v, X** dptr, hipStream_t s) {
  *dptr = nullptr;
  if (v.empty()) return MM_OK;
  void* p = nullptr;
  const size_t bytes = v.size() * sizeof(X);
  if (hipMalloc(&p, bytes) != hipSuccess) return fail(MM_E_NOMEM, "device allocation failed (plan tables)");
  pl->allocs.push_back(p);
  pl->bytes += bytes;
  if (hipMemcpyAsync(p, v.data(), bytes, hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(MM_E_HIP, "host to device copy failed");
  *dptr = (X*)p;
  return MM_OK;
}

mm_status plan_alloc(mm_plan_s* pl, size_t bytes, void** out) {
  void* p = nullptr;
  if (bytes == 0) bytes = 8;
  if (hipMalloc(&p, bytes) != hipSuccess) return fail(MM_E_NOMEM, "device allocation failed");
  pl->allocs.push_back(p);
  pl->bytes += bytes;
  *out = p;
  return MM_OK;
}

static size_t psi_elem_size(int kind) {
  switch (kind) {
    case MM_PSI_F64: return 8;
    case MM_PSI_F32: return 4;
    case MM_PSI_U16: return 2;
    default: return 0;
  }
}

// noise spectrum table (FP64 form), hit counts, weight blocks P^T T^-1 P, their inverses and the
// solvable mask; waits for the stream
static mm_status plan_precompute(mm_plan_s* pl, hipStream_t s) {
  DevPlan& P = pl->dp;
  if (P.spec) {
    hipError_t es = launch_spectrum(P, (double*)P.spec, s);
    if (es != hipSuccess) return fail(MM_E_HIP, std::string("spectrum kernel launch: ") + hipGetErrorString(es));
  }
  hipError_t e = launch_bin(P, BSRC_PLAN, nullptr, EPI_PLAN, nullptr, (double*)pl->d_solvable, pl->d_winv,
                            pl->d_hits, s);
  if (e != hipSuccess) return fail(MM_E_HIP, std::string("plan kernel launch: ") + hipGetErrorString(e));
  std::vector<uint8_t> sol(pl->npix);
  if (hipMemcpyAsync(sol.data(), pl->d_solvable, pl->npix, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(MM_E_HIP, std::string("plan precompute failed: ") + hipGetErrorString(hipGetLastError()));
  int64_t nsol = 0;
  for (int64_t i = 0; i < pl->npix; ++i) nsol += sol[i];
  pl->nsolvable = nsol;
  return MM_OK;
}

static bool noise_ok(double sg, double fk, double al, const double* tau, int64_t c, std::string& why) {
  if (!(sg > 0) || !(fk > 0) || !std::isfinite(al) || !std::isfinite(sg) || !std::isfinite(fk)) {
    why = "chunk " + std::to_string(c) + ": invalid noise parameters";
    return false;
  }
  if (tau && (!(tau[c] > 0) || tau[c] > sg * sg * (1 + 1e-12))) {
    why = "chunk " + std::to_string(c) + ": tau must satisfy 0 < tau <= sigma^2";
    return false;
  }
  return true;
}

mm_status plan_set_noise(mm_plan_s* pl, const double* sigma, const double* fknee, const double* alpha,
                         const double* tau, hipStream_t s) {
  if (!sigma || !fknee || !alpha) return fail(MM_E_ARG, "missing noise parameters");
  std::string why;
  for (int64_t c = 0; c < pl->nchunk; ++c)
    if (!noise_ok(sigma[c], fknee[c], alpha[c], tau, c, why)) return fail(MM_E_ARG, why);
  for (int64_t c = 0; c < pl->nchunk; ++c) {
    pl->sigma[c] = sigma[c];
    pl->fknee[c] = fknee[c];
    pl->alpha[c] = alpha[c];
    pl->tau[c] = tau ? tau[c] : sigma[c] * sigma[c];
    DevChunk& ch = pl->chunks_host[c];
    ch.sigma2 = sigma[c] * sigma[c];
    ch.fknee = fknee[c];
    ch.alpha = alpha[c];
    ch.tau = pl->tau[c];
    ch.inv_tau = 1.0 / ch.tau;
    ch.nbar0 = ch.sigma2 - ch.tau;
    ch.lg0 = std::log2(ch.df / ch.fknee);
  }
  if (hipMemcpyAsync(pl->d_chunks, pl->chunks_host.data(), pl->chunks_host.size() * sizeof(DevChunk),
                     hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(MM_E_HIP, "chunk table upload failed");
  mm_status st = plan_precompute(pl, s);
  if (st != MM_OK) return st;
  if (pl->nsolvable == 0) return fail(MM_E_SINGULAR, "no pixel has a solvable weight block");
  return MM_OK;
}

mm_status build_plan(const mm_plan_desc* desc, hipStream_t s, mm_plan_s** out) {
  if (!desc || !out) return fail(MM_E_ARG, "null descriptor or output");
  const mm_plan_desc& D = *desc;
  if (D.ncomp != 1 && D.ncomp != 3) return fail(MM_E_ARG, "ncomp must be 1 or 3");
  if (D.precision != MM_FP64 && D.precision != MM_MIXED) return fail(MM_E_ARG, "unknown precision");
  if (D.npix <= 0 || D.npix > (int64_t)INT32_MAX) return fail(MM_E_ARG, "npix out of range");
  if (D.nx < 0 || (D.nx > 0 && D.npix % D.nx != 0)) return fail(MM_E_ARG, "nx must divide npix");
  if (D.nchunk <= 0 || D.nchunk > (int64_t)INT32_MAX) return fail(MM_E_ARG, "nchunk out of range");
  if (!D.chunk_off || !D.fsample || !D.sigma || !D.fknee || !D.alpha || !D.pix)
    return fail(MM_E_ARG, "missing chunk table, noise parameters or pointing");
  if (D.ncomp == 3) {
    if (!D.psi || (D.psi_kind != MM_PSI_F64 && D.psi_kind != MM_PSI_F32 && D.psi_kind != MM_PSI_U16))
      return fail(MM_E_ARG, "I/Q/U maps need polarization angles");
    if (D.psi_kind == MM_PSI_U16 && (!D.psi_table || D.psi_table_len <= 0 || D.psi_table_len > 65536))
      return fail(MM_E_ARG, "uint16 angle indices need a host angle table of 1..65536 entries");
  }
  if (D.map_access != MM_MAP_AUTO && D.map_access != MM_MAP_GATHER && D.map_access != MM_MAP_PROJECTED)
    return fail(MM_E_ARG, "unknown map_access");
  const bool pick_mode = D.tune >= MM_TUNE_PICK0 && D.tune < MM_TUNE_PICK0 + 4096;
  if (D.tune != MM_TUNE_MEASURE && D.tune != MM_TUNE_STATIC && !pick_mode) return fail(MM_E_ARG, "unknown tune mode");
  if (D.binning != MM_BIN_SORTED && D.binning != MM_BIN_ATOMIC) return fail(MM_E_ARG, "unknown binning mode");
  if (D.chunk_off[0] != 0) return fail(MM_E_ARG, "chunk_off[0] must be 0");
  for (int64_t c = 0; c < D.nchunk; ++c) {
    const int64_t n = D.chunk_off[c + 1] - D.chunk_off[c];
    if (n <= 0) return fail(MM_E_ARG, "chunk offsets must increase");
    if (n % 2 != 0 || n < 2) return fail(MM_E_LEN, "chunk " + std::to_string(c) + ": length must be even");
    if (!five_smooth(n / 2))
      return fail(MM_E_LEN, "chunk " + std::to_string(c) + ": half length must factor into 2, 3 and 5");
    if (n / 2 > (1 << 24)) return fail(MM_E_LEN, "chunk " + std::to_string(c) + ": too long");
    const double sg = D.sigma[c], fk = D.fknee[c], al = D.alpha[c], fs = D.fsample[c];
    if (!(sg > 0) || !(fk > 0) || !std::isfinite(al) || !(fs > 0) || !std::isfinite(sg) || !std::isfinite(fk) ||
        !std::isfinite(fs))
      return fail(MM_E_ARG, "chunk " + std::to_string(c) + ": invalid noise parameters");
    if (D.tau) {
      const double t = D.tau[c];
      if (!(t > 0) || t > sg * sg * (1 + 1e-12))
        return fail(MM_E_ARG, "chunk " + std::to_string(c) + ": tau must satisfy 0 < tau <= sigma^2");
    }
  }
  const int64_t ns = D.chunk_off[D.nchunk];

  auto* pl = new mm_plan_s();
  std::unique_ptr<mm_plan_s, void (*)(mm_plan_s*)> guard(pl, [](mm_plan_s* p) { destroy_plan(p); });
  pl->ncomp = D.ncomp;
  pl->precision = D.precision;
  pl->psi_kind = D.ncomp == 3 ? D.psi_kind : MM_PSI_NONE;
  pl->npix = D.npix;
  pl->nx = D.nx;
  pl->nchunk = D.nchunk;
  pl->ns = ns;
  pl->off.assign(D.chunk_off, D.chunk_off + D.nchunk + 1);
  pl->sigma.assign(D.sigma, D.sigma + D.nchunk);
  pl->tau.resize(D.nchunk);
  pl->fsample.assign(D.fsample, D.fsample + D.nchunk);
  pl->fknee.assign(D.fknee, D.fknee + D.nchunk);
  pl->alpha.assign(D.alpha, D.alpha + D.nchunk);
  for (int64_t c = 0; c < D.nchunk; ++c) pl->tau[c] = D.tau ? D.tau[c] : D.sigma[c] * D.sigma[c];

  const bool f64 = D.precision == MM_FP64;
  const size_t csz = f64 ? sizeof(double2) : sizeof(float2);

  // ---- transform classes (one per distinct chunk length), twiddles, chunk table, work lists
  std::vector<double2> tw;
  std::vector<DevClass> classes;
  std::vector<DevChunk> chunks(D.nchunk);
  std::vector<int64_t> class_M;
  std::vector<int> class_cb;
  size_t lds_ac = 0, lds_b = 0, lds_g = 0;
  int64_t spec_total = 0;
  int64_t xwork = 0;  // complex values of the work buffers (chunk bases 16-aligned)
  for (int64_t c = 0; c < D.nchunk; ++c) {
    const int64_t n = D.chunk_off[c + 1] - D.chunk_off[c];
    const int64_t M = n / 2;
    int cls = -1;
    for (size_t i = 0; i < class_M.size(); ++i)
      if (class_M[i] == M) cls = (int)i;
    if (cls < 0) {
      const std::vector<Layout> cands = layout_candidates(M, f64);
      if (cands.empty())
        return fail(MM_E_LEN, "chunk " + std::to_string(c) + ": no transform split fits the LDS budget");
      int pick = 0;
      if (D.tune == MM_TUNE_MEASURE)
        pick = tune_layout(M, f64, cands, s);
      else if (D.tune >= MM_TUNE_PICK0)
        pick = std::min<int>(D.tune - MM_TUNE_PICK0, (int)cands.size() - 1);
      const Layout& L = cands[pick];
      DevClass k;
      make_class(M, L, tw, k);
      cls = (int)classes.size();
      classes.push_back(k);
      class_M.push_back(M);
      class_cb.push_back(L.cb);
      pl->class_layout.push_back(pick);
      pl->class_ncand.push_back((int32_t)cands.size());
      lds_b = std::max(lds_b, (size_t)((row_fuse(L.M1, f64) ? 4 : 2) * L.M1) * csz);
      lds_g = std::max(lds_g, (size_t)(4 * L.M1) * csz);  // rows of r and of P z
    }
    const DevClass& k = classes[cls];
    DevChunk& ch = chunks[c];
    std::memset(&ch, 0, sizeof(ch));
    ch.off = D.chunk_off[c];
    ch.n = (int32_t)n;
    ch.M = k.M;
    ch.M1 = k.M1;
    ch.M2 = k.M2;
    ch.cls = cls;
    ch.cb = (int32_t)class_cb[cls];
    ch.lgb = 0;
    while ((1 << (ch.lgb + 1)) <= ch.cb) ++ch.lgb;
    ch.df = D.fsample[c] / (double)n;
    ch.sigma2 = D.sigma[c] * D.sigma[c];
    ch.fknee = D.fknee[c];
    ch.alpha = D.alpha[c];
    ch.tau = pl->tau[c];
    ch.inv_tau = 1.0 / pl->tau[c];
    ch.nbar0 = ch.sigma2 - ch.tau;
    ch.spec_off = spec_total;
    ch.inv_M = 1.0 / (double)ch.M;
    ch.lg0 = std::log2(ch.df / ch.fknee);
    ch.xoff = xwork;
    xwork += (ch.M + kWorkAlign - 1) / kWorkAlign * kWorkAlign;
    spec_total += ch.M + 1;
    pl->chunk_item_begin.push_back((int32_t)pl->itemsB.size());
    pl->chunk_itemG_begin.push_back((int32_t)pl->itemsG.size());
    append_col_items((int32_t)c, ch, pl->itemsAC);
    append_row_items((int32_t)c, ch, pl->itemsB, row_fuse(ch.M1, f64));
    append_row_items((int32_t)c, ch, pl->itemsG, false);
  }
  pl->chunk_item_begin.push_back((int32_t)pl->itemsB.size());
  pl->chunk_itemG_begin.push_back((int32_t)pl->itemsG.size());
  bool all_pow2 = true;
  for (const DevClass& k : classes)
    for (int i = 0; i < k.nr1 + k.nr2; ++i) {
      const int r = i < k.nr1 ? k.rad1[i] : k.rad2[i - k.nr1];
      if (r != 2 && r != 4 && r != 8) all_pow2 = false;
    }
  // the inverse column pass takes the wave-local layout for every eligible class, except in
  // FP64 power-of-two plans (their inlined workgroup-wide stages measured faster)
  const bool wave_ok = !(f64 && all_pow2);
  size_t lds_c = 0;
  int nwave = 0;
  for (size_t i = 0; i < classes.size(); ++i) {
    const bool wl = wave_ok && wave_cols(classes[i].M2, class_cb[i], (int)csz);
    nwave += wl ? 1 : 0;
    lds_ac = std::max(lds_ac, (size_t)col_tile_elems(classes[i].M2, class_cb[i], (int)csz, false) * csz);
    lds_c = std::max(lds_c, (size_t)col_tile_elems(classes[i].M2, class_cb[i], (int)csz, wl) * csz);
  }
  pl->nwork = 2 * xwork;
  pl->lds_ac = lds_ac;
  pl->lds_c = lds_c;
  pl->lds_b = lds_b;
  pl->lds_g = lds_g;
  if (lds_c > (size_t)kMaxColTileBytes || lds_b + (kBlockB / 64) * sizeof(double) > 65536)
    return fail(MM_E_LEN, "transform tiles exceed the LDS budget");
  {
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      return fail(MM_E_HIP, "device LDS query failed");
    if (lds_c > (size_t)lds_max)
      return fail(MM_E_LEN, "column tiles of " + std::to_string(lds_c) + " bytes exceed the device's " +
                                std::to_string(lds_max) + " bytes of LDS per workgroup");
  }
  std::vector<float2> tw32(tw.size());
  for (size_t i = 0; i < tw.size(); ++i) tw32[i] = make_float2((float)tw[i].x, (float)tw[i].y);

  // ---- pointing: copy to host, validate, sort by pixel tile
  std::vector<int32_t> pix(ns);
  if (hipMemcpy(pix.data(), D.pix, ns * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(MM_E_HIP, "copying the pointing to the host failed (is pix a device pointer?)");
  for (int64_t j = 0; j < ns; ++j)
    if (pix[j] >= D.npix) return fail(MM_E_ARG, "pixel index " + std::to_string(pix[j]) + " beyond the map");
  const size_t pes = psi_elem_size(pl->psi_kind);
  std::vector<uint8_t> psi;
  if (pes) {
    psi.resize(ns * pes);
    if (hipMemcpy(psi.data(), D.psi, ns * pes, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(MM_E_HIP, "copying the angles to the host failed (is psi a device pointer?)");
    if (pl->psi_kind == MM_PSI_U16) {
      const uint16_t* ix = (const uint16_t*)psi.data();
      for (int64_t j = 0; j < ns; ++j)
        if (ix[j] >= D.psi_table_len) return fail(MM_E_ARG, "angle index beyond the table");
    } else {
      // the kernels' angle reduction is exact for |psi| < kMaxAngle
      for (int64_t j = 0; j < ns; ++j) {
        const double a = pl->psi_kind == MM_PSI_F64 ? ((const double*)psi.data())[j]
                                                    : (double)((const float*)psi.data())[j];
        if (!(std::fabs(a) < kMaxAngle)) return fail(MM_E_ARG, "angle " + std::to_string(j) + " is not finite or too large");
      }
    }
  }

  // tiles: rectangles of tw x th pixels over a map of rows of length nxm
  const int64_t nxm = D.nx > 0 ? D.nx : D.npix;
  const int64_t nym = D.npix / nxm;
  int64_t target = std::max<int64_t>(16, std::min<int64_t>(kMaxTilePix, D.npix / 2048));
  // Tile shape: about `target` pixels, tw a power of two, shaped by the scan.  A sample moving
  // (mx, my) pixels per step stays about 1 / (mx / tw + my / th) steps in a tile, so the shape
  // that maximises it gives the longest time-contiguous segments (fewer, longer HBM runs for
  // the staging reads and the P m writes).  mx, my: mean steps between consecutive on-map
  // samples of a chunk (every 4th pair; jumps of more than 16 pixels, such as scan-line
  // turnarounds, left out).
  double mx = 0.0, my = 0.0;
  {
    double sx = 0.0, sy = 0.0;
    int64_t nst = 0;
    for (int64_t c = 0; c < D.nchunk; ++c)
      for (int64_t j = D.chunk_off[c] + 1; j < D.chunk_off[c + 1]; j += 4) {
        const int32_t a = pix[j - 1], b = pix[j];
        if (a < 0 || b < 0) continue;
        const int64_t dx = std::llabs((int64_t)(b % nxm) - (a % nxm)), dy = std::llabs((int64_t)(b / nxm) - (a / nxm));
        if (dx > 16 || dy > 16) continue;
        sx += (double)dx;
        sy += (double)dy;
        ++nst;
      }
    mx = nst ? sx / (double)nst : 1.0;
    my = nst ? sy / (double)nst : 1.0;
    if (mx + my <= 0.0) mx = my = 1.0;
  }
  int64_t tw_ = 1, th_ = target;
  {
    double best = -1.0;
    for (int64_t w = 1; w <= std::min<int64_t>(target, nxm); w *= 2) {
      const int64_t h = std::min<int64_t>(nym, std::max<int64_t>(1, target / w));
      const double visit = 1.0 / (mx / (double)w + my / (double)h);
      if (visit > best * 1.000001) {
        best = visit;
        tw_ = w;
        th_ = h;
      }
    }
  }
  if (nym == 1) {
    tw_ = target;
    th_ = 1;
  }
  tw_ = std::min(tw_, nxm);
  th_ = std::min(th_, nym);
  const int64_t ntx = (nxm + tw_ - 1) / tw_, nty = (nym + th_ - 1) / th_;
  const int64_t ntiles = ntx * nty;
  std::vector<int64_t> tcount(ntiles + 1, 0);
  auto tile_of = [&](int32_t p) -> int64_t {
    const int64_t y = p / nxm, x = p % nxm;
    return (y / th_) * ntx + (x / tw_);
  };
  for (int64_t j = 0; j < ns; ++j)
    if (pix[j] >= 0) ++tcount[tile_of(pix[j]) + 1];
  for (int64_t t = 0; t < ntiles; ++t) tcount[t + 1] += tcount[t];
  const int64_t non = tcount[ntiles];
  std::vector<int64_t> order(non);
  {
    std::vector<int64_t> fill(tcount.begin(), tcount.end() - 1);
    for (int64_t j = 0; j < ns; ++j)
      if (pix[j] >= 0) order[fill[tile_of(pix[j])]++] = j;
  }
  // pixel-sorted arrays: every sub-batch starts on a kSortAlign-element boundary so that a lane
  // can fetch its run of consecutive entries with 16-byte loads; a tile of n samples has at most
  // ceil(n / kMaxSegs) sub-batches (each sub-batch holds kSubBatch samples or kMaxSegs segments)
  std::vector<int64_t> sbase(ntiles + 1, 0);
  for (int64_t t = 0; t < ntiles; ++t) {
    const int64_t cnt = tcount[t + 1] - tcount[t];
    const int64_t cap = cnt + kSortAlign * ((cnt + kMaxSegs - 1) / kMaxSegs + 1);
    sbase[t + 1] = sbase[t] + (cap + kSortAlign - 1) / kSortAlign * kSortAlign;
  }
  const int64_t nsorted = sbase[ntiles];
  std::vector<uint16_t> perm(nsorted, 0), lpv(nsorted, 0);
  std::vector<uint8_t> psi_sorted(nsorted * pes, 0);
  std::vector<Tile> tiles(ntiles);
  // per-tile sub-batches: consecutive runs of the tile's time-ordered samples holding at most
  // kSubBatch samples and kMaxSegs time-contiguous segments (segments never cross chunks)
  std::vector<std::vector<Segment>> tsegs(ntiles);
  std::vector<std::vector<SubBatch>> tsbs(ntiles);
  const std::vector<int64_t>& coff = pl->off;
  auto chunk_of = [&](int64_t j) -> int32_t {
    return (int32_t)(std::upper_bound(coff.begin(), coff.end(), j) - coff.begin() - 1);
  };
  std::atomic<int64_t> next(0);
  auto worker = [&]() {
    std::vector<int32_t> hist;
    for (;;) {
      const int64_t t = next.fetch_add(1);
      if (t >= ntiles) break;
      const int64_t ty = t / ntx, tx = t % ntx;
      Tile tl;
      tl.x0 = (int32_t)(tx * tw_);
      tl.y0 = (int32_t)(ty * th_);
      tl.tw = (int32_t)std::min(tw_, nxm - tx * tw_);
      tl.th = (int32_t)std::min(th_, nym - ty * th_);
      tl.sb_begin = tl.sb_end = 0;
      tiles[t] = tl;
      const int64_t tp = (int64_t)tl.tw * tl.th;
      hist.assign(tp + 1, 0);
      auto lp_of = [&](int64_t j) -> int32_t {
        const int64_t p = pix[j];
        const int64_t y = p / nxm, x = p % nxm;
        return (int32_t)((y - tl.y0) * tl.tw + (x - tl.x0));
      };
      std::vector<Segment>& sg = tsegs[t];
      int64_t i = tcount[t];
      const int64_t iend = tcount[t + 1];
      int64_t cursor = sbase[t];
      while (i < iend) {
        SubBatch S;
        S.sorted_begin = cursor;
        S.seg_begin = (int32_t)sg.size();
        S.pad = 0;
        const int64_t b0 = i;
        int64_t cur_end = -1;
        int64_t chunk_end = -1;
        int nseg = 0;
        for (; i < iend && i - b0 < kSubBatch; ++i) {
          const int64_t j = order[i];
          if (!(j == cur_end && j < chunk_end)) {
            if (nseg == kMaxSegs) break;
            Segment g;
            g.start = j;
            g.pos = (int32_t)(i - b0);
            g.chunk = chunk_of(j);
            chunk_end = coff[g.chunk + 1];
            sg.push_back(g);
            ++nseg;
          }
          cur_end = j + 1;
        }
        const int64_t b1 = i;
        S.count = (int32_t)(b1 - b0);
        S.seg_end = (int32_t)sg.size();
        // counting sort of the sub-batch by local pixel (stable: time order within a pixel)
        std::fill(hist.begin(), hist.end(), 0);
        for (int64_t q = b0; q < b1; ++q) ++hist[lp_of(order[q]) + 1];
        for (int64_t l = 0; l < tp; ++l) hist[l + 1] += hist[l];
        for (int64_t q = b0; q < b1; ++q) {
          const int64_t j = order[q];
          const int32_t l = lp_of(j);
          const int64_t dst = cursor + hist[l]++;
          perm[dst] = (uint16_t)(q - b0);
          lpv[dst] = (uint16_t)l;
          if (pes) std::memcpy(&psi_sorted[dst * pes], &psi[j * pes], pes);
        }
        tsbs[t].push_back(S);
        cursor += (S.count + kSortAlign - 1) / kSortAlign * kSortAlign;
      }
    }
  };
  {
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (unsigned i = 0; i < nth; ++i) th.emplace_back(worker);
    for (auto& x : th) x.join();
  }
  std::vector<SubBatch> sbs;
  std::vector<Segment> segs;
  for (int64_t t = 0; t < ntiles; ++t) {
    const int32_t base = (int32_t)segs.size();
    tiles[t].sb_begin = (int32_t)sbs.size();
    for (SubBatch S : tsbs[t]) {
      S.seg_begin += base;
      S.seg_end += base;
      sbs.push_back(S);
    }
    tiles[t].sb_end = (int32_t)sbs.size();
    segs.insert(segs.end(), tsegs[t].begin(), tsegs[t].end());
    std::vector<Segment>().swap(tsegs[t]);
    std::vector<SubBatch>().swap(tsbs[t]);
  }
  pl->ntiles = ntiles;
  pl->nsegs = (int64_t)segs.size();
  pl->tile_w = (int32_t)tw_;
  pl->tile_h = (int32_t)th_;

  // ---- device uploads
  DevPlan& P = pl->dp;
  std::memset(&P, 0, sizeof(P));
  P.ncomp = D.ncomp;
  P.all_pow2 = all_pow2 ? 1 : 0;
  P.max_tile_pix = (int32_t)(tw_ * th_);
  P.col_wave = nwave == 0 ? 0 : (nwave == (int)classes.size() ? 1 : 2);
  P.psi_kind = pl->psi_kind;
  P.precision = D.precision;
  P.npix = D.npix;
  P.nxm = nxm;
  P.nsamp = ns;
  P.nchunk = (int32_t)D.nchunk;
  P.ntiles = (int32_t)ntiles;
  P.pix = D.pix;
  P.psi = D.psi;
  mm_status st;
  DevChunk* dchunks;
  DevClass* dclasses;
  double2* dtw64;
  float2* dtw32;
  if ((st = upload(pl, chunks, &dchunks, s)) != MM_OK) return st;
  pl->chunks_host = chunks;
  pl->d_chunks = dchunks;
  if ((st = upload(pl, classes, &dclasses, s)) != MM_OK) return st;
  if ((st = upload(pl, tw, &dtw64, s)) != MM_OK) return st;
  if ((st = upload(pl, tw32, &dtw32, s)) != MM_OK) return st;
  P.chunks = dchunks;
  P.classes = dclasses;
  P.tw64 = dtw64;
  P.tw32 = dtw32;
  {
    std::vector<double2> sc(1024);
    for (int k = 0; k < 1024; ++k) {
      const double a = M_PI * (double)k / 512.0;
      sc[k] = make_double2(std::cos(a), std::sin(a));
    }
    double2* dsc;
    if ((st = upload(pl, sc, &dsc, s)) != MM_OK) return st;
    P.sc_tab = dsc;
  }
  if (pl->psi_kind == MM_PSI_U16) {
    std::vector<double2> cs64(D.psi_table_len);
    std::vector<float2> cs32(D.psi_table_len);
    for (int64_t i = 0; i < D.psi_table_len; ++i) {
      const double a = 2.0 * (double)D.psi_table[i];
      if (!(std::fabs(a) < 2.0 * kMaxAngle)) return fail(MM_E_ARG, "angle table entry is not finite or too large");
      cs64[i] = make_double2(std::cos(a), std::sin(a));
      cs32[i] = make_float2((float)cs64[i].x, (float)cs64[i].y);
    }
    double2* d64;
    float2* d32;
    if ((st = upload(pl, cs64, &d64, s)) != MM_OK) return st;
    if ((st = upload(pl, cs32, &d32, s)) != MM_OK) return st;
    P.psi_cs64 = d64;
    P.psi_cs32 = d32;
  }
  Tile* dtiles;
  SubBatch* dsbs;
  Segment* dsegs;
  uint16_t *dperm, *dlp;
  uint8_t* dpsis = nullptr;
  if ((st = upload(pl, tiles, &dtiles, s)) != MM_OK) return st;
  if ((st = upload(pl, sbs, &dsbs, s)) != MM_OK) return st;
  if ((st = upload(pl, segs, &dsegs, s)) != MM_OK) return st;
  if ((st = upload(pl, perm, &dperm, s)) != MM_OK) return st;
  if ((st = upload(pl, lpv, &dlp, s)) != MM_OK) return st;
  if (pes && (st = upload(pl, psi_sorted, &dpsis, s)) != MM_OK) return st;
  P.tiles = dtiles;
  P.sbs = dsbs;
  P.segs = dsegs;
  P.perm = dperm;
  P.lp = dlp;
  P.psi_sorted = dpsis;
  if ((st = upload(pl, pl->itemsAC, &pl->d_itemsAC, s)) != MM_OK) return st;
  if ((st = upload(pl, pl->itemsB, &pl->d_itemsB, s)) != MM_OK) return st;
  if ((st = upload(pl, pl->chunk_item_begin, &pl->d_chunk_item_begin, s)) != MM_OK) return st;
  if ((st = upload(pl, pl->itemsG, &pl->d_itemsG, s)) != MM_OK) return st;
  if ((st = upload(pl, pl->chunk_itemG_begin, &pl->d_chunk_itemG_begin, s)) != MM_OK) return st;

  const int64_t mapn = (int64_t)D.ncomp * D.npix;
  const int nw = D.ncomp == 1 ? 1 : 6;
  void* p;
  if ((st = plan_alloc(pl, (size_t)nw * D.npix * sizeof(double), &p)) != MM_OK) return st;
  pl->d_winv = (double*)p;
  if ((st = plan_alloc(pl, (size_t)D.npix, &p)) != MM_OK) return st;
  pl->d_solvable = (uint8_t*)p;
  if ((st = plan_alloc(pl, (size_t)D.npix * sizeof(int32_t), &p)) != MM_OK) return st;
  pl->d_hits = (int32_t*)p;
  if ((st = plan_alloc(pl, (size_t)pl->nwork * (f64 ? 8 : 4), &p)) != MM_OK) return st;
  pl->d_work = p;
  if ((st = plan_alloc(pl, std::max(pl->itemsB.size(), 3 * pl->itemsG.size()) * sizeof(double), &p)) != MM_OK)
    return st;
  pl->d_chi2_part = (double*)p;  // chi^2 partials (1 per row item) or gradient partials (3 per item)
  if ((st = plan_alloc(pl, 64 * sizeof(double), &p)) != MM_OK) return st;
  pl->d_scal = (double*)p;
  if ((st = plan_alloc(pl, 1024 * sizeof(double), &p)) != MM_OK) return st;
  pl->d_part = (double*)p;
  for (int i = 0; i < kScratchMaps; ++i) {
    if ((st = plan_alloc(pl, (size_t)mapn * sizeof(double), &p)) != MM_OK) return st;
    pl->d_map[i] = (double*)p;
  }
  P.winv = pl->d_winv;
  P.solvable = pl->d_solvable;
  if (f64) {
    if ((st = plan_alloc(pl, (size_t)spec_total * sizeof(double), &p)) != MM_OK) return st;
    P.spec = (double*)p;
  }
  // maps larger than the L2 of one XCD (4 MB) are gathered badly by the strided column pass:
  // then P m is produced in pixel-tile order instead
  pl->pm_mode = D.map_access == MM_MAP_PROJECTED ||
                (D.map_access == MM_MAP_AUTO && mapn * (int64_t)sizeof(double) > ((int64_t)4 << 20));
  pl->bin_atomic = D.binning == MM_BIN_ATOMIC;
  for (int64_t c = 0; c < D.nchunk; ++c) pl->max_n = std::max<int64_t>(pl->max_n, D.chunk_off[c + 1] - D.chunk_off[c]);
  if (pl->bin_atomic) {
    if ((st = plan_alloc(pl, (size_t)mapn * sizeof(double), &p)) != MM_OK) return st;
    pl->d_batom = (double*)p;
  }
  if (!pl->pm_mode && D.ncomp == 3) {
    if ((st = plan_alloc(pl, (size_t)D.npix * 2 * sizeof(double2), &p)) != MM_OK) return st;
    P.mapi = (double2*)p;
  }
  if (pl->pm_mode) {
    if ((st = plan_alloc(pl, (size_t)ns * (f64 ? 8 : 4), &p)) != MM_OK) return st;
    pl->d_pm = p;
    if (hipMemsetAsync(p, 0, (size_t)ns * (f64 ? 8 : 4), s) != hipSuccess)  // off-map samples: P m = 0
      return fail(MM_E_HIP, "clearing the projection buffer failed");
  }
  if ((st = plan_precompute(pl, s)) != MM_OK) return st;
  if (pl->nsolvable == 0) return fail(MM_E_SINGULAR, "no pixel has a solvable weight block");
  if (hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return fail(MM_E_HIP, "stream creation failed");
  *out = guard.release();
  return MM_OK;
}

void destroy_plan(mm_plan_s* pl) {
  if (!pl) return;
  if (pl->solve_exec || !pl->allocs.empty()) (void)hipDeviceSynchronize();
  if (pl->solve_exec) (void)hipGraphExecDestroy(pl->solve_exec);
  if (pl->solve_done) (void)hipEventDestroy(pl->solve_done);
  for (auto& r : pl->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : pl->ev_pool) (void)hipEventDestroy(e);
  for (void* p : pl->allocs) (void)hipFree(p);
  for (void* p : pl->extra_allocs) (void)hipFree(p);
  if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
  delete pl;
}

}  // namespace mm
