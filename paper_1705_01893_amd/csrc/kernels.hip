// HIP kernels of the messenger-field mapmaking sweep (gfx950).
//
// One iteration of eqn. (mcompact), m <- m + W^-1 P^T (lambda^-1 N-bar + T)^-1 (d - P m),
// runs as four passes over the time-ordered data of every chunk (Section 2.1 lists
// the same cost centres: projection, forward transform, spectral filter, inverse
// transform, back-projection):
//
//   pass A  gather P m, residual r = d - P m, M2-point column transforms of the
//           complex sequence z_j = r_2j + i r_2j+1 (j = j1 + M1 j2), twiddle
//           omega_M^(j1 k2), write in row layout X[k2 * M1 + j1];
//   pass B  per pair of rows {k2, M2 - k2}: M1-point row transforms give Z_k
//           (k = k2 + M2 k1); the partner bin M - k lives in the paired row, so the
//           real spectrum R_k, R_{M-k} is untangled in registers, multiplied by the
//           noise filter (and summed into chi^2), re-tangled, inverse-transformed
//           along the rows and twiddled back;
//   pass C  inverse column transforms: y = G r in time order, in place;
//   pass D  deterministic binning P^T y per pixel tile, fused with the per-pixel
//           3x3 solve and map update.
//
// All passes use one TOD-sized work buffer in place.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "common.h"
#include "fft.h"

namespace mm {

// ---------------------------------------------------------------------------------------------
// small helpers

static inline int grid_for(int64_t n, int cap) { return (int)(n < cap ? (n > 0 ? n : 1) : cap); }
constexpr int kGridCap = 1 << 16;

template <typename T>
__device__ __forceinline__ const cx<T>* twtab(const DevPlan& P);
template <>
__device__ __forceinline__ const float2* twtab<float>(const DevPlan& P) { return P.tw32; }
template <>
__device__ __forceinline__ const double2* twtab<double>(const DevPlan& P) { return P.tw64; }

// omega_{2M}^q = exp(-2 pi i q / (2M)), 0 <= q < 2M, from the two-level table: tw + twhi holds
// omega_2M^(h 2^lb), tw + twlo omega_2M^rem (rem < 2^lb)
template <typename T>
__device__ __forceinline__ cx<T> omega2M_tab(const cx<T>* tw, int64_t twhi, int64_t twlo, int lb, int q) {
  return cmul(tw[twhi + (q >> lb)], tw[twlo + (q & ((1 << lb) - 1))]);
}

template <typename T>
__device__ __forceinline__ cx<T> omega2M(const DevPlan& P, const DevClass& cl, int q) {
  return omega2M_tab<T>(twtab<T>(P), cl.twhi, cl.twlo, cl.lb, q);
}

// omega_{2M}^(q0 + u dq) for u = 0..U-1, with 0 <= q0, dq < 2M: one table lookup pair for the
// start and one for the step instead of a lookup pair per element, the step's powers by
// balanced products (s^u = (s^(u/2))^2 or s^(u-1) s), so that the rounding grows like log2 u
// ulps.  Used by the FP32 transforms, where the lookups' memory round trips cost more than the
// products; the FP64 form keeps its per-element lookups (it has no registers to spare).
template <typename T, int U>
__device__ __forceinline__ void omega2M_run_tab(const cx<T>* tw, int64_t twhi, int64_t twlo, int lb, int q0, int dq,
                                                cx<T>* w) {
  const cx<T> w0 = omega2M_tab<T>(tw, twhi, twlo, lb, q0);
  w[0] = w0;
  if constexpr (U > 1) {
    const cx<T> st = omega2M_tab<T>(tw, twhi, twlo, lb, dq);
    cx<T> pw[U];
    pw[1] = st;
    w[1] = cmul(w0, st);
#pragma unroll
    for (int u = 2; u < U; ++u) {
      pw[u] = (u % 2 == 0) ? cmul(pw[u / 2], pw[u / 2]) : cmul(pw[u - 1], st);
      w[u] = cmul(w0, pw[u]);
    }
  }
}

template <typename T, int U>
__device__ __forceinline__ void omega2M_run(const DevPlan& P, const DevClass& cl, int q0, int dq, cx<T>* w) {
  omega2M_run_tab<T, U>(twtab<T>(P), cl.twhi, cl.twlo, cl.lb, q0, dq, w);
}

template <typename C>
__device__ __forceinline__ C conjc(C a) {
  a.y = -a.y;
  return a;
}

// sin and cos of an angle in float64: theta = k pi/512 + r with |r| <= pi/1024 (Cody-Waite
// reduction with a two-part constant; the fused multiply-adds keep k times the leading part
// exact), tabulated (cos, sin)(k pi/512), Taylor series of sin r and cos r (the first omitted
// terms are below 2e-19 relative), and the angle-sum formulas.  Exact reduction needs
// |theta| < 2 kMaxAngle, which the plan checks for every stored angle.
__device__ __forceinline__ void sincos_tab(const double2* __restrict__ tab, double th, double& s, double& c) {
  const double kf = rint(th * 162.97466172610083);          // 512 / pi
  double r = fma(-kf, 0.006135923151542565, th);            // pi/512, leading part
  r = fma(-kf, 2.391888279584674e-19, r);                   // pi/512, trailing part
  const double2 t = tab[(int)kf & 1023];
  const double r2 = r * r;
  const double sr = r * fma(r2, fma(r2, fma(r2, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0), 1.0);
  const double cr = fma(r2, fma(r2, fma(r2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
  c = fma(t.x, cr, -t.y * sr);
  s = fma(t.y, cr, t.x * sr);
}

// sin and cos of an angle in float64 without memory accesses: theta = k pi/2 + r, |r| <= pi/4
// (Cody-Waite reduction with a three-part pi/2; the fused multiply-adds keep k times each part
// exact for the angles the plan admits), Taylor series of sin r to r^17 and of cos r to r^18
// (truncation below 5e-17) by Horner's rule, and the quadrant's signs and swap.  Within
// 1.4e-16 of the exact values on a host check over |theta| < 2e5.
__device__ __forceinline__ void sincos_q(double th, double& s, double& c) {
  const double kf = rint(th * 0.6366197723675814);  // 2/pi
  double r = fma(-kf, 1.5707963267948966, th);
  r = fma(-kf, 6.123233995736766e-17, r);
  r = fma(-kf, -1.4973849048591698e-33, r);
  const double r2 = r * r;
  double ps = 1.0 / 355687428096000.0;
  ps = fma(ps, r2, -1.0 / 1307674368000.0);
  ps = fma(ps, r2, 1.0 / 6227020800.0);
  ps = fma(ps, r2, -1.0 / 39916800.0);
  ps = fma(ps, r2, 1.0 / 362880.0);
  ps = fma(ps, r2, -1.0 / 5040.0);
  ps = fma(ps, r2, 1.0 / 120.0);
  ps = fma(ps, r2, -1.0 / 6.0);
  const double sr = fma(r * r2, ps, r);
  double pc = 1.0 / 6402373705728000.0;
  pc = fma(pc, r2, -1.0 / 20922789888000.0);
  pc = fma(pc, r2, 1.0 / 87178291200.0);
  pc = fma(pc, r2, -1.0 / 479001600.0);
  pc = fma(pc, r2, 1.0 / 3628800.0);
  pc = fma(pc, r2, -1.0 / 40320.0);
  pc = fma(pc, r2, 1.0 / 720.0);
  pc = fma(pc, r2, -1.0 / 24.0);
  pc = fma(pc, r2, 0.5);
  const double cr = fma(-r2, pc, 1.0);
  const int q = (int)kf & 3;
  const double ss = (q & 1) ? cr : sr, cc = (q & 1) ? sr : cr;
  s = (q & 2) ? -ss : ss;
  c = ((q + 1) & 2) ? -cc : cc;
}

// The same in float32, for the FP32-mixed form: three-part pi/2 (the fused multiply-adds keep
// the reduction's error near one rounding of r for the angles the plan admits), Taylor series of
// sin r to r^9 and of cos r to r^8 (truncation below 1e-8 for |r| <= pi/4).  Within 9.5e-8 of
// the exact values (1.6 units in the last place at 1) on a host check over |theta| < 2e5; the
// library sincosf reaches 7e-8 there but carries a large-argument path the stored angles never
// need.
__device__ __forceinline__ void sincos_qf(float th, float& s, float& c) {
  const float kf = rintf(th * 0.636619747f);  // 2/pi
  float r = fmaf(-kf, 1.57079637f, th);
  r = fmaf(-kf, -4.37113883e-08f, r);
  r = fmaf(-kf, -1.71512451e-15f, r);
  const float r2 = r * r;
  float ps = fmaf(r2, 1.0f / 362880.0f, -1.0f / 5040.0f);
  ps = fmaf(r2, ps, 1.0f / 120.0f);
  ps = fmaf(r2, ps, -1.0f / 6.0f);
  const float sr = fmaf(r * r2, ps, r);
  float pc = fmaf(r2, 1.0f / 40320.0f, -1.0f / 720.0f);
  pc = fmaf(r2, pc, 1.0f / 24.0f);
  pc = fmaf(r2, pc, -0.5f);
  const float cr = fmaf(r2, pc, 1.0f);
  const int q = (int)kf & 3;
  const float ss = (q & 1) ? cr : sr, cc = (q & 1) ? sr : cr;
  s = (q & 2) ? -ss : ss;
  c = ((q + 1) & 2) ? -cc : cc;
}

// polarization weights (cos 2psi, sin 2psi) of one stored angle, computed in the TOD precision
template <typename T>
__device__ __forceinline__ void psi_weights(const DevPlan& P, const void* arr, int64_t i, T& c, T& s);

template <>
__device__ __forceinline__ void psi_weights<double>(const DevPlan& P, const void* arr, int64_t i, double& c,
                                                    double& s) {
  if (P.psi_kind == 1) {
    sincos_q(2.0 * ((const double*)arr)[i], s, c);
  } else if (P.psi_kind == 2) {
    sincos_q(2.0 * (double)((const float*)arr)[i], s, c);
  } else {
    const double2 t = P.psi_cs64[((const uint16_t*)arr)[i]];
    c = t.x;
    s = t.y;
  }
}
template <>
__device__ __forceinline__ void psi_weights<float>(const DevPlan& P, const void* arr, int64_t i, float& c,
                                                   float& s) {
  if (P.psi_kind == 1) {
    const float a = (float)(2.0 * ((const double*)arr)[i]);
    sincos_qf(a, s, c);
  } else if (P.psi_kind == 2) {
    const float a = 2.0f * ((const float*)arr)[i];
    sincos_qf(a, s, c);
  } else {
    const float2 t = P.psi_cs32[((const uint16_t*)arr)[i]];
    c = t.x;
    s = t.y;
  }
}

// (P m)_j for one sample (float64)
// noise spectrum pieces at real bin k: pl = sigma^2 (f/fknee)^alpha with the DC bin at f_1
template <typename T>
__device__ __forceinline__ T powerlaw(const DevChunk& ch, int k);
template <>
__device__ __forceinline__ double powerlaw<double>(const DevChunk& ch, int k) {
  const double f = (double)(k == 0 ? 1 : k) * ch.df;
  return ch.sigma2 * pow(f / ch.fknee, ch.alpha);
}
template <>
__device__ __forceinline__ float powerlaw<float>(const DevChunk& ch, int k) {
  // sigma^2 2^(alpha (log2 k + log2(df / fknee))) with the hardware base-2 log and exponential
  const float lk = __builtin_amdgcn_logf((float)(k == 0 ? 1 : k));
  return (float)ch.sigma2 * __builtin_amdgcn_exp2f((float)ch.alpha * (lk + (float)ch.lg0));
}

struct BinCtx {
  int gain, chi2;
  double lam, inv_lam, chi2_lam;
  double* modes;  // per-mode chi^2 terms of the launch's chunk, indexed by real bin k (or null)
};

// power-law part sigma^2 (f_k/fknee)^alpha of the noise spectrum at real bin k: tabulated at plan
// time in the FP64 form, evaluated in single precision in the FP32-mixed form.  The table is in
// row layout: bin k = k2 + M2 k1 sits at k2 * M1 + k1 (bin M last), so a row of the transform
// reads a contiguous run; tidx is that position (the row pass knows it without dividing).
template <typename T>
__device__ __forceinline__ T powerlaw_bin(const DevPlan& P, const DevChunk& ch, int k, int tidx);
template <>
__device__ __forceinline__ double powerlaw_bin<double>(const DevPlan& P, const DevChunk& ch, int k, int tidx) {
  return P.spec[ch.spec_off + tidx];
}
template <>
__device__ __forceinline__ float powerlaw_bin<float>(const DevPlan& P, const DevChunk& ch, int k, int tidx) {
  return powerlaw<float>(ch, k);
}

__device__ __forceinline__ int spec_index(const DevChunk& ch, int k) {
  return (k == ch.M) ? ch.M : (k % ch.M2) * ch.M1 + k / ch.M2;
}

// 1/x: correctly rounded in float64; the hardware reciprocal (1 ulp) in float32
template <typename T>
__device__ __forceinline__ T recip(T x);
template <>
__device__ __forceinline__ double recip<double>(double x) {
  return 1.0 / x;
}
template <>
__device__ __forceinline__ float recip<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}

// gain applied to R_k (includes the 1/M of the inverse transform) and chi^2 weight 1/(n N'_k)
template <typename T>
__device__ __forceinline__ void bin_factors_pl(const DevChunk& ch, const BinCtx& bc, T pl, T& g, double& cw) {
  const T N = (T)ch.sigma2 + pl;
  const T tau = (T)ch.tau;
  T gg;
  if (bc.gain == GAIN_MESSENGER) {
    const T nbar = (T)ch.nbar0 + pl;
    gg = recip<T>(tau + nbar * (T)bc.inv_lam);
  } else if (bc.gain == GAIN_MESSENGER_PL) {
    gg = recip<T>(tau + pl * (T)bc.inv_lam);
  } else if (bc.gain == GAIN_GAPFILL) {
    const T eps = (T)ch.nbar0;  // sigma^2 - tau
    gg = eps * recip<T>(eps + pl);
  } else if (bc.gain == GAIN_NINV) {
    gg = recip<T>(N);
  } else {
    gg = N * (T)ch.inv_tau;
  }
  g = gg * (T)ch.inv_M;
  // chi^2 weight 1 / (n N'_k), N' = N + (lambda - 1) tau, in the TOD precision, only when asked for
  cw = 0.0;
  if (bc.chi2) cw = (double)recip<T>((T)ch.n * (N + (T)((bc.chi2_lam - 1.0) * ch.tau)));
}

template <typename T>
__device__ __forceinline__ void bin_factors(const DevPlan& P, const DevChunk& ch, const BinCtx& bc, int k, int tidx,
                                            T& g, double& cw) {
  bin_factors_pl<T>(ch, bc, powerlaw_bin<T>(P, ch, k, tidx), g, cw);
}

template <typename C>
__device__ __forceinline__ double norm2(C a) {
  return (double)a.x * (double)a.x + (double)a.y * (double)a.y;
}

// ---------------------------------------------------------------------------------------------
// pass A: residual + column transforms

// angle pair of samples 2ci, 2ci+1 (one vector load) -> weights in the TOD precision
template <typename T>
struct PsiPair {
  T c0, s0, c1, s1;
};

template <typename T>
__device__ __forceinline__ void psi_pair_load(const DevPlan& P, int pk, int64_t ci, uint4& raw) {
  if (pk == 1) {
    const double2 v = ((const double2*)P.psi)[ci];
    raw.x = __double2loint(v.x);
    raw.y = __double2hiint(v.x);
    raw.z = __double2loint(v.y);
    raw.w = __double2hiint(v.y);
  } else if (pk == 2) {
    const float2 v = ((const float2*)P.psi)[ci];
    raw.x = __float_as_uint(v.x);
    raw.y = __float_as_uint(v.y);
  } else {
    raw.x = ((const uint32_t*)P.psi)[ci];
  }
}

template <typename T>
__device__ __forceinline__ void psi_from_raw(const DevPlan& P, int pk, const uint4& raw, int which, T& c, T& s) {
  if (pk == 1) {
    const double a = which == 0 ? __hiloint2double(raw.y, raw.x) : __hiloint2double(raw.w, raw.z);
    if (sizeof(T) == 8) {
      double sd, cd;
      sincos_tab(P.sc_tab, 2.0 * a, sd, cd);
      c = (T)cd;
      s = (T)sd;
    } else {
      float sf, cf;
      sincos_qf((float)(2.0 * a), sf, cf);
      c = (T)cf;
      s = (T)sf;
    }
  } else if (pk == 2) {
    const float a = __uint_as_float(which == 0 ? raw.x : raw.y);
    if (sizeof(T) == 8) {
      double sd, cd;
      sincos_tab(P.sc_tab, 2.0 * (double)a, sd, cd);
      c = (T)cd;
      s = (T)sd;
    } else {
      float sf, cf;
      sincos_qf(2.0f * a, sf, cf);
      c = (T)cf;
      s = (T)sf;
    }
  } else {
    const uint32_t idx = which == 0 ? (raw.x & 0xffffu) : (raw.x >> 16);
    if (sizeof(T) == 8) {
      const double2 t = P.psi_cs64[idx];
      c = (T)t.x;
      s = (T)t.y;
    } else {
      const float2 t = P.psi_cs32[idx];
      c = (T)t.x;
      s = (T)t.y;
    }
  }
}

// Item order of the column passes.  Workgroups are dispatched to the 8 XCDs round-robin by
// index, and adjacent column blocks of a chunk share 128-byte lines: a block's run in each row
// starts wherever the row does (rows of M1 complex values), and in FP64 adjacent blocks share
// the lines of the 8-byte pixel pairs.  Within each group of kXcd * kXcdRun workgroups, XCD x
// takes the kXcdRun consecutive items x kXcdRun, ..., so that most shared lines are fetched by
// one L2.  A bijection of every full group; the launch rounds the grid up to whole groups
// (other grids keep the plain order).
constexpr int kXcd = 8, kXcdRun = 8;
constexpr int kGroupNoGather = 16;  // loads issued together per thread in the forward column pass, no gather
__host__ __device__ inline int col_grid(int64_t nitems) {
  constexpr int g = kXcd * kXcdRun;
  const int64_t n = (nitems + g - 1) / g * g;
  return (int)(n < kGridCap ? (n > 0 ? n : g) : kGridCap);
}
// wave-uniform values in scalar registers: a work item's sizes and offsets, read once, so that
// per-element address arithmetic does not wait on the vector loads that fetched them
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni64(int64_t x) {
  const uint32_t lo = (uint32_t)uni((int)(uint32_t)x), hi = (uint32_t)uni((int)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int xcd_run_order(int b, int grid) {
  constexpr int g = kXcd * kXcdRun;
  if (grid % g) return b;
  const int r = b & (g - 1);
  return (b - r) + (r % kXcd) * kXcdRun + r / kXcd;
}

// NG: the source needs no map gather (d, P m from its buffer, or their difference).  PK: the
// angles of the gather form, fixed at compile time so that no run-time branch on them separates
// the loads (0 none: temperature only; 1 float64, 2 float32, 3 uint16 table index; -1: not used)
// X2 (no-gather sources only): a second TOD stream read beside the first, P_B m of composite
// pointing or d_0 and the gap flags of gap filling (kept out of the plain variants' registers).
template <typename T, bool P2, bool NG, int PK, bool X2 = false>
__global__ __launch_bounds__(kBlock, 4) void k_pass_a(DevPlan P, const ItemAC* __restrict__ items, int nitems,
                                                   const T* __restrict__ d, const double* __restrict__ m, int src,
                                                   cx<T>* __restrict__ X, const T* __restrict__ pmbuf) {
  constexpr int E = Ept<T>::v;
  // elements whose loads are issued together: all of them without a gather, else 4 (the
  // gather's pixel, angle and map values take registers)
  constexpr int G = NG ? (kGroupNoGather < E ? kGroupNoGather : E) : (sizeof(T) == 8 && PK > 0 ? 2 : 4);
  constexpr int pk = PK;
  constexpr int nc = PK == 0 ? 1 : 3;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  for (int it = xcd_run_order(blockIdx.x, gridDim.x); it < nitems; it += gridDim.x) {
    const ItemAC item = items[it];
    const DevChunk ch = P.chunks[item.chunk];
    const DevClass& cl = P.classes[ch.cls];
    const int B = uni(ch.cb), lgB = uni(ch.lgb), M1 = uni(ch.M1), M2 = uni(ch.M2);
    const int j10 = uni(item.j1);
    const int nbv = min(B, M1 - j10);
    const int ntot = B * M2;
    const int64_t cbase = uni64(ch.off) / 2 + j10;
#pragma unroll 1
    for (int g = 0; g < E; g += G) {
      int2 pp[G];
      constexpr int G2 = X2 ? G : 1;
      cx<T> dd[G], pb[G], pb2[G2];
      uint16_t gf[G2];
      uint4 raw[G];
      bool ok[G];
      // every load of the group goes out before any is used: elements outside the item read the
      // item's first pair (a valid address) and are discarded, so no per-element branch separates
      // the loads
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int e = threadIdx.x + (g + u) * kBlock;
        const int b = e & (B - 1), j2 = e >> lgB;
        ok[u] = (e < ntot) && (b < nbv);
        const int64_t ci = ok[u] ? cbase + b + (int64_t)M1 * j2 : cbase;
        pp[u] = make_int2(-1, -1);
        dd[u].x = T(0);
        dd[u].y = T(0);
        pb[u].x = T(0);
        pb[u].y = T(0);
        if constexpr (X2) {
          pb2[u].x = T(0);
          pb2[u].y = T(0);
          gf[u] = 0;
        }
        if (src != SRC_PM && src != SRC_PMBUF) dd[u] = ((const cx<T>*)d)[ci];
        if (src == SRC_PMBUF || src == SRC_D_MINUS_PMBUF) {
          pb[u] = ((const cx<T>*)pmbuf)[ci];
          if constexpr (X2) pb2[u] = ((const cx<T>*)pmbuf)[ci + P.pmb_off];  // composite: P_B m
        } else if (X2 && src == SRC_GAP) {
          if constexpr (X2) {
            pb[u] = ((const cx<T>*)pmbuf)[ci];      // t_0
            pb2[u] = ((const cx<T>*)P.gap_d0)[ci];  // d_0
            gf[u] = ((const uint16_t*)P.gaps)[ci];  // the pair's two gap flags
          }
        } else if (!NG && src != SRC_D) {
          const int2 q = ((const int2*)P.pix)[ci];
          pp[u] = ok[u] ? q : make_int2(-1, -1);
          if (nc == 3) psi_pair_load<T>(P, pk, ci, raw[u]);
        }
      }
      double pm[G][2];
#pragma unroll
      for (int u = 0; u < G; ++u) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          // flagged samples (px < 0) read pixel 0 and are discarded: no branch between the gathers
          const int px = h == 0 ? pp[u].x : pp[u].y;
          const int pc = px >= 0 ? px : 0;
          double v;
          if (nc == 3) {
            // the interleaved copy: I, Q and U of a pixel share one cache line
            const double2 iq = P.mapi[2 * pc], u0 = P.mapi[2 * pc + 1];
            T c, sn;
            psi_from_raw<T>(P, pk, raw[u], h, c, sn);
            v = iq.x + (double)c * iq.y + (double)sn * u0.x;
          } else {
            v = m[pc];
          }
          pm[u][h] = px >= 0 ? v : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int e = threadIdx.x + (g + u) * kBlock;
        if (e < ntot) {
          cx<T> z;
          if (!ok[u]) {
            z.x = T(0);
            z.y = T(0);
          } else if (src == SRC_D) {
            z = dd[u];
          } else if (!NG && src == SRC_PM) {
            z.x = (T)pm[u][0];
            z.y = (T)pm[u][1];
          } else if (src == SRC_PMBUF) {
            z = pb[u];
            if constexpr (X2) {
              z.x = (T)((double)pb[u].x + (double)pb2[u].x);
              z.y = (T)((double)pb[u].y + (double)pb2[u].y);
            }
          } else if (src == SRC_D_MINUS_PMBUF) {
            double px = (double)pb[u].x, py = (double)pb[u].y;
            if constexpr (X2) {
              px += (double)pb2[u].x;
              py += (double)pb2[u].y;
            }
            z.x = (T)((double)dd[u].x - px);
            z.y = (T)((double)dd[u].y - py);
          } else if (X2 && src == SRC_GAP) {
            // t_0 - t_1, t_1 = d outside the gaps, d_0 inside
            if constexpr (X2) {
              z.x = (T)((double)pb[u].x - (double)((gf[u] & 0xffu) ? pb2[u].x : dd[u].x));
              z.y = (T)((double)pb[u].y - (double)((gf[u] >> 8) ? pb2[u].y : dd[u].y));
            }
          } else if (!NG) {
            z.x = (T)((double)dd[u].x - pm[u][0]);
            z.y = (T)((double)dd[u].y - pm[u][1]);
          }
          lds[e] = z;
        }
      }
    }
    __syncthreads();
    lds_transform<T, false, true, kBlock, P2>(lds, M2, B, lgB, cl.rad2, cl.nr2, twtab<T>(P) + cl.tw2);
    cx<T>* Xc = X + uni64(ch.xoff);
    // the four-step twiddles omega_2M^(2 j1 k2).  kBlock is a multiple of the block width, so a
    // thread keeps its column b and its elements step k2 by S = kBlock / B: along each half of
    // them the twiddles form a geometric run (elements outside the item take the q = 0 start
    // and store nothing)
    const int bq = threadIdx.x & (B - 1), k20 = threadIdx.x >> lgB, S = kBlock >> lgB;
    const int jj = j10 + bq;
    const int dq = (S < M2 && bq < nbv) ? 2 * jj * S : 0;
#pragma unroll 1
    for (int h = 0; h < E; h += E / 2) {
      const int k2h = k20 + h * S;
      cx<T> w[E / 2];
      if constexpr (X2 || sizeof(T) == 8) {
        // the two-stream variants and the FP64 form keep one lookup pair per element (the runs
        // would spill the former's registers and measured slower in the latter): the table
        // offsets read once, the lookups issued together
        const cx<T>* tw = twtab<T>(P);
        const int64_t twhi = uni64(cl.twhi), twlo = uni64(cl.twlo);
        const int lb = uni(cl.lb);
#pragma unroll
        for (int u = 0; u < E / 2; ++u) {
          const int e = threadIdx.x + (h + u) * kBlock;
          const int b = e & (B - 1), k2 = e >> lgB;
          const int q = (e < ntot && b < nbv) ? 2 * (j10 + b) * k2 : 0;
          w[u] = cmul(tw[twhi + (q >> lb)], tw[twlo + (q & ((1 << lb) - 1))]);
        }
      } else {
        omega2M_run<T, E / 2>(P, cl, (k2h < M2 && bq < nbv) ? 2 * jj * k2h : 0, dq, w);
      }
#pragma unroll
      for (int u = 0; u < E / 2; ++u) {
        const int e = threadIdx.x + (h + u) * kBlock;
        const int b = e & (B - 1), k2 = e >> lgB;
        if (e < ntot && b < nbv) Xc[(int64_t)k2 * M1 + j10 + b] = cmul(lds[e], w[u]);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// pass B: row transforms, real-spectrum untangle, filter, chi^2, retangle, inverse rows

template <typename T>
__device__ __forceinline__ void b_pair(cx<T>* lds, const DevPlan& P, const DevChunk& ch, const DevClass& cl,
                                       const BinCtx& bc, int ops, int k, int ia, int ib, T plk, T plm,
                                       double& chi, const cx<T>* wpre = nullptr) {
  // bins k (LDS ia, power law plk) and M - k (LDS ib, power law plm); wpre: omega_2M^k when the
  // caller has fetched it already
  const cx<T> Zk = lds[ia], Zm = lds[ib];
  cx<T> E, O;
  E.x = T(0.5) * (Zk.x + Zm.x);
  E.y = T(0.5) * (Zk.y - Zm.y);
  // O = (Zk - conj(Zm)) / (2i)
  O.x = T(0.5) * (Zk.y + Zm.y);
  O.y = -T(0.5) * (Zk.x - Zm.x);
  const cx<T> w = wpre ? *wpre : omega2M<T>(P, cl, k);
  const cx<T> wO = cmul(w, O);
  const cx<T> Rk = cadd(E, wO);
  const cx<T> Rm = csub(conjc(E), conjc(wO));
  T gk, gm;
  double cwk, cwm;
  bin_factors_pl<T>(ch, bc, plk, gk, cwk);
  bin_factors_pl<T>(ch, bc, plm, gm, cwm);
  if (ops & B_CHI2) chi += 2.0 * (norm2(Rk) * cwk + norm2(Rm) * cwm);
  if (bc.modes) {
    bc.modes[k] = 2.0 * norm2(Rk) * cwk;
    bc.modes[ch.M - k] = 2.0 * norm2(Rm) * cwm;
  }
  if (ops & B_FILTER) {
    const cx<T> Yk = cscale(Rk, gk), Ym = cscale(Rm, gm);
    cx<T> Ep, D;
    Ep.x = T(0.5) * (Yk.x + Ym.x);
    Ep.y = T(0.5) * (Yk.y - Ym.y);
    D.x = T(0.5) * (Yk.x - Ym.x);
    D.y = T(0.5) * (Yk.y + Ym.y);
    const cx<T> Op = cmul(D, conjc(w));
    // Z'_k = E' + i O',  Z'_{M-k} = conj(E') + i conj(O')
    cx<T> zk, zm;
    zk.x = Ep.x - Op.y;
    zk.y = Ep.y + Op.x;
    zm.x = Ep.x + Op.y;
    zm.y = -Ep.y + Op.x;
    lds[ia] = zk;
    lds[ib] = zm;
  }
}

template <typename T>
__device__ __forceinline__ void b_dc(cx<T>* lds, const DevPlan& P, const DevChunk& ch, const BinCtx& bc, int ops,
                                     int ia, double& chi) {
  const cx<T> Z = lds[ia];
  const T R0 = Z.x + Z.y, RM = Z.x - Z.y;
  T g0, gM;
  double c0, cM;
  bin_factors<T>(P, ch, bc, 0, 0, g0, c0);
  bin_factors<T>(P, ch, bc, ch.M, ch.M, gM, cM);
  if (ops & B_CHI2) chi += (double)R0 * (double)R0 * c0 + (double)RM * (double)RM * cM;
  if (bc.modes) {
    bc.modes[0] = (double)R0 * (double)R0 * c0;
    bc.modes[ch.M] = (double)RM * (double)RM * cM;
  }
  if (ops & B_FILTER) {
    const T Y0 = R0 * g0, YM = RM * gM;
    cx<T> z;
    z.x = T(0.5) * (Y0 + YM);
    z.y = T(0.5) * (Y0 - YM);
    lds[ia] = z;
  }
}

template <typename T>
__device__ __forceinline__ void b_self(cx<T>* lds, const DevPlan& P, const DevChunk& ch, const BinCtx& bc, int ops,
                                       int k, int ia, int ta, double& chi) {
  // k = M/2: R_k = conj(Z_k); the retangled value is conj(Y_k)
  const cx<T> Z = lds[ia];
  T g;
  double cw;
  bin_factors<T>(P, ch, bc, k, ta, g, cw);
  if (ops & B_CHI2) chi += 2.0 * norm2(Z) * cw;
  if (bc.modes) bc.modes[k] = 2.0 * norm2(Z) * cw;
  if (ops & B_FILTER) {
    cx<T> y;
    y.x = Z.x * g;
    y.y = Z.y * g;  // conj(conj(Z) g)
    lds[ia] = y;
  }
}

// Rows of a row item between the work buffer and LDS (row r at r * M1).  NR: rows the item may
// hold (2: one pair or a self-paired row, nrow <= 2; 4: two pairs); NR * M1 <= kBlockB * Ept.
// FP32: every load of a thread is issued before the first LDS write (one memory round trip per
// item, not one per element); slots past the row end or the item's rows read element 0 of the
// chunk, a valid address, and are not stored.  FP64 keeps the per-element form, which measured
// faster there.
template <typename T, int NR>
__device__ __forceinline__ void row_load(cx<T>* lds, const cx<T>* __restrict__ Xc, const int* rws, int nrow, int M1) {
  constexpr int U = Ept<T>::v / NR;
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = threadIdx.x + u * kBlockB;
      if (e < M1) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (r < nrow) lds[r * M1 + e] = Xc[(int64_t)rws[r] * M1 + e];
      }
    }
    return;
  }
  cx<T> v[U][NR];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = threadIdx.x + u * kBlockB;
#pragma unroll
    for (int r = 0; r < NR; ++r) v[u][r] = Xc[(e < M1 && r < nrow) ? (int64_t)rws[r] * M1 + e : 0];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = threadIdx.x + u * kBlockB;
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (e < M1 && r < nrow) lds[r * M1 + e] = v[u][r];
  }
}

// the inverse row transforms' output, times the conjugate column twiddle, back to the work buffer;
// FP32: each row's twiddles from a geometric run, formed before the stores (slots past the row
// end or the item's rows take the q = 0 run and store nothing)
template <typename T, int NR>
__device__ __forceinline__ void row_store(const cx<T>* lds, cx<T>* __restrict__ Xc, const DevPlan& P,
                                          const DevClass& cl, const int* rws, int nrow, int M1) {
  constexpr int U = Ept<T>::v / NR;
  // along a row r, a thread's elements j1 = t + u kBlockB have the twiddles omega_2M^(2 r j1):
  // a geometric run from omega^(2 r t) in steps of omega^(2 r kBlockB)
  // (the FP64 form keeps a lookup pair per element)
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j1 = threadIdx.x + u * kBlockB;
      if (j1 < M1) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (r < nrow) Xc[(int64_t)rws[r] * M1 + j1] = cmul(lds[r * M1 + j1], conjc(omega2M<T>(P, cl, 2 * j1 * rws[r])));
      }
    }
    return;
  }
  const bool tok = (int)threadIdx.x < M1;
  const int dstep = (tok && kBlockB < M1) ? 2 * kBlockB : 0;
  cx<T> w[U][NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const bool ok = r < nrow && tok;
    cx<T> wr[U];
    omega2M_run<T, U>(P, cl, ok ? 2 * (int)threadIdx.x * rws[r] : 0, ok ? dstep * rws[r] : 0, wr);
#pragma unroll
    for (int u = 0; u < U; ++u) w[u][r] = wr[u];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j1 = threadIdx.x + u * kBlockB;
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (j1 < M1 && r < nrow) Xc[(int64_t)rws[r] * M1 + j1] = cmul(lds[r * M1 + j1], conjc(w[u][r]));
  }
}

// Pairs of rows under the precision's compiled-in schedule (FP32: 2048 points, radices 8, 16, 16;
// FP64: 1024 points, radices 4, 4, 8, 8) touch the work buffer from their first and last stages
// directly, without the row load's and the row store's passes through LDS.
//
// First forward stage (radix R, p = 1, L / R butterflies per row, one per thread): butterfly k
// of row b takes elements k + (L / R) m (m < R) of work row b, the elements the row load would
// have put in its LDS inputs, and writes its outputs to LDS as the LDS stage does.
template <typename T, int L, int R>
__device__ __attribute__((noinline)) void row_first_from_work(cx<T>* lds_generic, const cx<T>* x0_generic,
                                                              const cx<T>* x1_generic) {
  constexpr int NBF = L / R;
  static_assert(NBF == kBlockB, "one butterfly of each row per thread");
  const lds_v2<T> lds = (lds_v2<T>)lds_generic;
  const glob_v2<T> x0 = (glob_v2<T>)x0_generic, x1 = (glob_v2<T>)x1_generic;
  const int k = (int)threadIdx.x;
  cx<T> v[2][R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    v[0][m] = to_cx<T>(x0[k + m * NBF]);
    v[1][m] = to_cx<T>(x1[k + m * NBF]);
  }
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    Dft<T, R, false>::run(v[b]);
#pragma unroll
    for (int m = 0; m < R; ++m) lds[b * L + k * R + m] = to_v2<T>(v[b][m]);
  }
  __syncthreads();
}

// Last inverse stage (radix R, p = P = L / R, so that its twiddle step L / (P R) is 1): thread t
// takes butterfly j = t mod P of row b = t / P, whose outputs are the row's elements
// j1 = j + P m; each goes to work row r_b times the conjugate column twiddle omega_2M^(-2 r_b j1)
// (a geometric run in m, in FP64 too: a lookup pair per element needs registers this stage does
// not have), as the row store would have written it.  No LDS writes follow, so no barrier.
template <typename T, int L, int R>
__device__ __attribute__((noinline)) void row_last_to_work(const cx<T>* lds_generic, cx<T>* x0_generic,
                                                           cx<T>* x1_generic, int r0, int r1,
                                                           const cx<T>* __restrict__ tw1, const cx<T>* tw,
                                                           int64_t twhi, int64_t twlo, int lb) {
  constexpr int P = L / R, NBF = L / R;
  static_assert(2 * NBF == kBlockB, "one butterfly per thread");
  const lds_v2<T> lds = (lds_v2<T>)lds_generic;
  const int b = (int)threadIdx.x / NBF, j = (int)threadIdx.x % NBF;
  cx<T> v[R];
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = to_cx<T>(lds[b * L + j + m * NBF]);
  if (j != 0) {
    cx<T> w = to_cx<T>(((glob_v2<T>)tw1)[j]);
    w.y = -w.y;
    twiddle_powers<T, R>(v, w);
  }
  Dft<T, R, true>::run(v);
  const int r = b ? r1 : r0;
  using globw_v2 = __attribute__((address_space(1))) vec2<T>*;
  const globw_v2 x = (globw_v2)(b ? x1_generic : x0_generic);
  cx<T> wr[R];
  omega2M_run_tab<T, R>(tw, twhi, twlo, lb, 2 * j * r, 2 * P * r, wr);
#pragma unroll
  for (int m = 0; m < R; ++m) x[j + m * P] = to_v2<T>(cmul(v[m], conjc(wr[m])));
}

// the compiled-in schedules, forward from the work buffer into LDS and inverse from LDS into the
// work buffer
template <typename T>
__device__ __forceinline__ void row_ct_forward_from_work(cx<T>* lds, const cx<T>* x0, const cx<T>* x1,
                                                         const cx<T>* __restrict__ tw1) {
  if constexpr (sizeof(T) == 4) {
    row_first_from_work<T, 2048, 8>(lds, x0, x1);
    stage_ct<T, 16, false, 2048, 2, 8, kBlockB>(lds, tw1);
    stage_ct<T, 16, false, 2048, 2, 128, kBlockB>(lds, tw1);
  } else {
    row_first_from_work<T, 1024, 4>(lds, x0, x1);
    stage_ct<T, 4, false, 1024, 2, 4, kBlockB>(lds, tw1);
    stage_ct<T, 8, false, 1024, 2, 16, kBlockB>(lds, tw1);
    stage_ct<T, 8, false, 1024, 2, 128, kBlockB>(lds, tw1);
  }
}

template <typename T>
__device__ __forceinline__ void row_ct_inverse_to_work(cx<T>* lds, cx<T>* x0, cx<T>* x1, int r0, int r1,
                                                       const cx<T>* __restrict__ tw1, const cx<T>* tw,
                                                       int64_t twhi, int64_t twlo, int lb) {
  if constexpr (sizeof(T) == 4) {
    stage_ct<T, 8, true, 2048, 2, 1, kBlockB>(lds, tw1);
    stage_ct<T, 16, true, 2048, 2, 8, kBlockB>(lds, tw1);
    row_last_to_work<T, 2048, 16>(lds, x0, x1, r0, r1, tw1, tw, twhi, twlo, lb);
  } else {
    stage_ct<T, 4, true, 1024, 2, 1, kBlockB>(lds, tw1);
    stage_ct<T, 4, true, 1024, 2, 4, kBlockB>(lds, tw1);
    stage_ct<T, 8, true, 1024, 2, 16, kBlockB>(lds, tw1);
    row_last_to_work<T, 1024, 8>(lds, x0, x1, r0, r1, tw1, tw, twhi, twlo, lb);
  }
}

// at most 128 VGPRs, so that four 256-thread workgroups share a CU
template <typename T>
__global__ __launch_bounds__(kBlockB, 4) void k_pass_b(DevPlan P, const ItemB* __restrict__ items, int nitems,
                                                   cx<T>* __restrict__ X, int ops, BinCtx bc,
                                                   double* __restrict__ chi2_part, int red_off) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  double* red = reinterpret_cast<double*>(smem_raw + red_off);
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const ItemB item = items[it];
    const DevChunk ch = P.chunks[item.chunk];
    const DevClass& cl = P.classes[ch.cls];
    const int M1 = ch.M1, M2 = ch.M2;
    const int ra = item.ra, rb = item.rb, rc = item.rc;
    // LDS rows: ra, rb, then (two pairs) rc, M2 - rc
    const int nrow = rc > 0 ? 4 : ((ra == rb) ? 1 : 2);
    cx<T>* Xc = X + ch.xoff;
    const int rws[4] = {ra, rb, rc, M2 - rc};
    const cx<T>* tw1 = twtab<T>(P) + cl.tw1;
    // pairs of rows under the precision's compiled-in radix schedule: stages specialised at
    // compile time, the first and last of them reading and writing the work buffer
    const bool ct = row_ct_ok<T>(M1, nrow, cl.nr1, cl.rad1);
    if (ct) {
      row_ct_forward_from_work<T>(lds, Xc + (int64_t)ra * M1, Xc + (int64_t)rb * M1, tw1);
    } else {
      if (rc > 0)
        row_load<T, 4>(lds, Xc, rws, 4, M1);
      else
        row_load<T, 2>(lds, Xc, rws, nrow, M1);
      __syncthreads();
      lds_fft<T, false, false, kBlockB>(lds, M1, nrow, 0, cl.rad1, cl.nr1, tw1);
    }
    double chi = 0.0;
    const bool self_a = (ra == 0) || (2 * ra == M2);
    if (!self_a) {
      // one or two pairs of rows (r, M2 - r): bins k = r + M2 k1 and M - k = (M2 - r) + M2 (M1 - 1 - k1),
      // at most E/2 steps per thread.  The FP64 form reads the power law from its table: all of
      // a thread's values are fetched first, so that their latencies overlap.
      const int nt = (rc > 0 ? 2 : 1) * M1;
      if constexpr (sizeof(T) == 8) {
        constexpr int U = Ept<T>::v / 2;
        T plk[U], plm[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int t = threadIdx.x + u * kBlockB;
          const int q = t >= M1 ? 1 : 0;
          const int k1 = t - q * M1, pk1 = M1 - 1 - k1;
          const int r = q ? rc : ra, rr = M2 - r;
          if (t < nt) {
            plk[u] = powerlaw_bin<T>(P, ch, r + M2 * k1, r * M1 + k1);
            plm[u] = powerlaw_bin<T>(P, ch, ch.M - (r + M2 * k1), rr * M1 + pk1);
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int t = threadIdx.x + u * kBlockB;
          const int q = t >= M1 ? 1 : 0;
          const int k1 = t - q * M1, pk1 = M1 - 1 - k1;
          if (t < nt)
            b_pair<T>(lds, P, ch, cl, bc, ops, (q ? rc : ra) + M2 * k1, 2 * q * M1 + k1, (2 * q + 1) * M1 + pk1,
                      plk[u], plm[u], chi);
        }
      } else {
        // the FP32-mixed form evaluates the power law in place; the twiddle reads of all of a
        // thread's bins go out first
        constexpr int U = Ept<T>::v / 2;
        cx<T> wk[U];
        if (M1 == U * kBlockB || (rc > 0 && 2 * M1 == U * kBlockB)) {
          // one row of U elements per thread, or two rows of U/2: bins k = r + M2 (t + u kBlockB)
          // along each row, a geometric run in steps of omega_2M^(M2 kBlockB)
          const int dq = M2 * kBlockB;
          if (M1 == U * kBlockB) {
            omega2M_run<T, U>(P, cl, ra + M2 * (int)threadIdx.x, dq, wk);
          } else {
            omega2M_run<T, U / 2>(P, cl, ra + M2 * (int)threadIdx.x, dq, wk);
            omega2M_run<T, U / 2>(P, cl, rc + M2 * (int)threadIdx.x, dq, wk + U / 2);
          }
        } else {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int t = threadIdx.x + u * kBlockB;
            const int q = t >= M1 ? 1 : 0;
            const int k1 = t - q * M1;
            wk[u] = omega2M<T>(P, cl, t < nt ? (q ? rc : ra) + M2 * k1 : 0);
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int t = threadIdx.x + u * kBlockB;
          if (t < nt) {
            const int q = t >= M1 ? 1 : 0;
            const int k1 = t - q * M1, pk1 = M1 - 1 - k1;
            const int r = q ? rc : ra, rr = M2 - r;
            const int k = r + M2 * k1;
            b_pair<T>(lds, P, ch, cl, bc, ops, k, 2 * q * M1 + k1, (2 * q + 1) * M1 + pk1,
                      powerlaw_bin<T>(P, ch, k, r * M1 + k1), powerlaw_bin<T>(P, ch, ch.M - k, rr * M1 + pk1), chi,
                      &wk[u]);
          }
        }
      }
    } else {
      for (int sl = 0; sl < nrow; ++sl) {
        const int row = sl == 0 ? ra : rb;
        for (int k1 = threadIdx.x; k1 < M1; k1 += kBlockB) {
          const int pk1 = (row == 0) ? (k1 == 0 ? 0 : M1 - k1) : (M1 - 1 - k1);
          if (k1 > pk1) continue;
          const int k = row + M2 * k1;
          // bins k and M - k both lie in this row (row 0 or row M2/2)
          if (k == 0)
            b_dc<T>(lds, P, ch, bc, ops, sl * M1, chi);
          else if (k1 == pk1)
            b_self<T>(lds, P, ch, bc, ops, k, sl * M1 + k1, row * M1 + k1, chi);
          else
            b_pair<T>(lds, P, ch, cl, bc, ops, k, sl * M1 + k1, sl * M1 + pk1,
                      powerlaw_bin<T>(P, ch, k, row * M1 + k1), powerlaw_bin<T>(P, ch, ch.M - k, row * M1 + pk1), chi);
        }
      }
    }
    if (ops & B_CHI2) {
      // fixed-order reduction: butterfly within each wave, then the waves in order
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) chi += __shfl_xor(chi, o);
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = chi;
      __syncthreads();
      if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlockB / 64; ++w) t += red[w];
        chi2_part[it] = t;
      }
    }
    if (ops & B_FILTER) {
      __syncthreads();
      if (ct) {
        row_ct_inverse_to_work<T>(lds, Xc + (int64_t)ra * M1, Xc + (int64_t)rb * M1, ra, rb, tw1, twtab<T>(P),
                                  cl.twhi, cl.twlo, cl.lb);
      } else {
        lds_fft<T, true, false, kBlockB>(lds, M1, nrow, 0, cl.rad1, cl.nr1, tw1);
        if (rc > 0)
          row_store<T, 4>(lds, Xc, P, cl, rws, 4, M1);
        else
          row_store<T, 2>(lds, Xc, P, cl, rws, nrow, M1);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// pass C: inverse column transforms -> filtered TOD in time order (in place)

// Blocks of NB interleaved FP64 columns of 2048 points under the radix schedule 4, 8, 8, 8 (the
// first candidate order for 2048-point FP64 columns): the stages specialised at compile time, the
// first reading the work buffer and the last writing it, without the load's and the store's
// passes through LDS.  Column b of the block is work column j10 + b (xc points at its row 0);
// element i sits at LDS slot i NB + b.
template <typename T, int L, int R, int NB>
__device__ __attribute__((noinline)) void col_first_from_work(cx<T>* lds_generic, const cx<T>* xc_generic, int M1) {
  constexpr int NBF = L / R, K = NBF * NB / kBlock;
  static_assert(NBF * NB == K * kBlock, "whole butterflies per thread");
  const lds_v2<T> lds = (lds_v2<T>)lds_generic;
  const glob_v2<T> x = (glob_v2<T>)xc_generic;
  cx<T> v[K][R];
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int f = (int)threadIdx.x + u * kBlock, b = f % NB, k = f / NB;
#pragma unroll
    for (int m = 0; m < R; ++m) v[u][m] = to_cx<T>(x[(int64_t)(k + m * NBF) * M1 + b]);
  }
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int f = (int)threadIdx.x + u * kBlock, b = f % NB, k = f / NB;
    Dft<T, R, true>::run(v[u]);
#pragma unroll
    for (int m = 0; m < R; ++m) lds[(k * R + m) * NB + b] = to_v2<T>(v[u][m]);
  }
  __syncthreads();
}

// the last stage (p = L / R, twiddle step 1): butterfly j of column b writes elements j + p m
template <typename T, int L, int R, int NB>
__device__ __attribute__((noinline)) void col_last_to_work(const cx<T>* lds_generic, cx<T>* xc_generic, int M1,
                                                           const cx<T>* __restrict__ tw2) {
  constexpr int P = L / R, NBF = L / R;
  static_assert(NBF * NB == kBlock, "one butterfly per thread");
  const lds_v2<T> lds = (lds_v2<T>)lds_generic;
  using globw_v2 = __attribute__((address_space(1))) vec2<T>*;
  const globw_v2 x = (globw_v2)xc_generic;
  const int b = (int)threadIdx.x % NB, j = (int)threadIdx.x / NB;
  cx<T> v[R];
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = to_cx<T>(lds[(j + m * NBF) * NB + b]);
  if (j != 0) {
    cx<T> w = to_cx<T>(((glob_v2<T>)tw2)[j]);
    w.y = -w.y;
    twiddle_powers<T, R>(v, w);
  }
  Dft<T, R, true>::run(v);
#pragma unroll
  for (int m = 0; m < R; ++m) x[(int64_t)(j + m * P) * M1 + b] = to_v2<T>(v[m]);
}

template <typename T>
__device__ __forceinline__ bool col_ct_ok(int M2, int B, int nbv, int nr, const int8_t* rad) {
  return sizeof(T) == 8 && M2 == 2048 && B == 2 && nbv == B && nr == 4 && rad[0] == 4 && rad[1] == 8 &&
         rad[2] == 8 && rad[3] == 8;
}

// WL: the LDS layout of the plan's classes: 0 interleaved (every class), 1 wave-local (every
// class), 2 each class's own (eligible ones wave-local), 3 wave-local with every class a
// 1024-point FP32 column per wave, transformed in registers.  At most 128 VGPRs: two 512-thread
// workgroups per CU.
template <typename T, bool P2, int WL>
__global__ __launch_bounds__(kBlock, 4) void k_pass_c(DevPlan P, const ItemAC* __restrict__ items, int nitems,
                                                   cx<T>* __restrict__ X) {
  constexpr int E = Ept<T>::v;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  for (int it = xcd_run_order(blockIdx.x, gridDim.x); it < nitems; it += gridDim.x) {
    const ItemAC item = items[it];
    const DevChunk ch = P.chunks[item.chunk];
    const DevClass& cl = P.classes[ch.cls];
    const int B = ch.cb, lgB = ch.lgb, M1 = ch.M1, M2 = ch.M2;
    const int j10 = item.j1;
    const int nbv = min(B, M1 - j10);
    const int ntot = B * M2;
    // per transform class: the wave-local layout where it is eligible (never with the inlined
    // power-of-two stages)
    const bool wl = !P2 && (WL == 1 || WL == 3 || (WL == 2 && wave_cols(M2, B, (int)sizeof(cx<T>))));
    const int Lc = wl ? wave_col_stride(M2, B, (int)sizeof(cx<T>)) : 0;
    cx<T>* Xc = X + ch.xoff + j10;
    if constexpr (sizeof(T) == 8) {
      if (!wl && col_ct_ok<T>(M2, B, nbv, cl.nr2, cl.rad2)) {
        const cx<T>* tw2 = twtab<T>(P) + cl.tw2;
        col_first_from_work<T, 2048, 4, 2>(lds, Xc, M1);
        stage_ct<T, 8, true, 2048, 2, 4, kBlock, true>(lds, tw2);
        stage_ct<T, 8, true, 2048, 2, 32, kBlock, true>(lds, tw2);
        col_last_to_work<T, 2048, 8, 2>(lds, Xc, M1, tw2);
        __syncthreads();
        continue;
      }
    }
    {
      cx<T> v[E];
#pragma unroll
      for (int u = 0; u < E; ++u) {
        const int e = threadIdx.x + u * kBlock;
        const int b = e & (B - 1), k2 = e >> lgB;
        v[u].x = T(0);
        v[u].y = T(0);
        if (e < ntot && b < nbv) v[u] = Xc[(int64_t)k2 * M1 + b];
      }
#pragma unroll
      for (int u = 0; u < E; ++u) {
        const int e = threadIdx.x + u * kBlock;
        if (e < ntot) lds[wl ? (e & (B - 1)) * Lc + pad8(e >> lgB) : e] = v[u];
      }
    }
    __syncthreads();
    if (wl) {
      if constexpr (WL == 3 && sizeof(T) == 4) {
        // every class: one 1024-point column per wave, transformed in registers (lane shuffles
        // between its radix-2 levels), back to the column in natural order
        wave_col1024_regs<true>(lds + (int)(threadIdx.x >> 6) * Lc, twtab<T>(P) + cl.tw2);
      } else {
        const int nw = B / kColWaves;
        wave_fft<T, true>(lds + (int)(threadIdx.x >> 6) * nw * Lc, M2, Lc, nw, cl.rad2, cl.nr2, twtab<T>(P) + cl.tw2);
      }
      __syncthreads();
    } else {
      lds_transform<T, true, true, kBlock, P2>(lds, M2, B, lgB, cl.rad2, cl.nr2, twtab<T>(P) + cl.tw2);
    }
    // the store addresses are formed here, not ahead of the transform calls (where they would
    // have to survive the calls in registers)
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
#pragma unroll
    for (int u = 0; u < E; ++u) {
      const int e = tid + u * kBlock;
      const int b = e & (B - 1), j2 = e >> lgB;
      if (e < ntot && b < nbv) Xc[(int64_t)M1 * j2 + b] = lds[wl ? b * Lc + pad8(j2) : e];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// pass D: deterministic binning per pixel tile (+ fused map update / plan precompute)
//
// One workgroup per tile.  For each sub-batch of the tile's samples:
//   1. the sub-batch's segment table goes to LDS and every thread stages its share of the
//      samples (time order) into LDS, locating each position's segment by binary search;
//   2. each wave owns a contiguous stripe of the sub-batch in pixel-sorted order, preloaded
//      into registers before the staging barrier; per 64-sample step it forms the
//      contributions, runs a segmented inclusive scan over equal pixels and adds each
//      completed run once to the LDS accumulator of its pixel.  The run that opens a stripe
//      may continue the previous stripe, so it is parked in a per-wave slot and added after a
//      barrier, in wave order: the summation order is fixed, hence bitwise reproducible.

template <typename T, int NV>
__device__ __forceinline__ void contrib(const DevPlan& P, double y, double c, double s, double* v) {
  if (NV == 1) {
    v[0] = y;
  } else if (NV == 3) {
    v[0] = y;
    v[1] = c * y;
    v[2] = s * y;
  } else if (NV == 2) {  // plan, temperature: hits, sum 1/tau
    v[0] = 1.0;
    v[1] = y;
  } else {  // NV == 7, plan, I/Q/U: hits and the six entries of sum a a^T / tau
    v[0] = 1.0;
    v[1] = y;
    v[2] = c * y;
    v[3] = s * y;
    v[4] = c * c * y;
    v[5] = c * s * y;
    v[6] = s * s * y;
  }
}

template <int NV>
__device__ __forceinline__ void bin_flush(double* acc, double* cv, int* clp, int wave, int lp, int first_lp,
                                          const double* v) {
  if (lp == first_lp) {
    clp[wave] = lp;
#pragma unroll
    for (int q = 0; q < NV; ++q) cv[wave * NV + q] = v[q];
  } else {
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[lp * NV + q] += v[q];
  }
}

// Staging position -> segment of one sub-batch.  Positions [0, count) are split into
// time-contiguous segments; segment i starts at position spos[i] (spos[0] = 0).  A bitmap in LDS
// marks the starts (bit q & 63 of word q >> 6).  Lane l of each wave keeps word l and the index of
// the segment holding position 64 l (a prefix count of the starts), so a lookup costs three lane
// reads and a popcount instead of a search.
struct SegIndex {
  uint32_t lo, hi;
  int base;
};

__device__ __forceinline__ SegIndex seg_index(const unsigned long long* smask) {
  const int lane = threadIdx.x & 63;
  const unsigned long long w = smask[lane];
  const int n = __popcll(w);
  int s = n;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(s, d);
    if (lane >= d) s += t;
  }
  SegIndex r;
  r.lo = (uint32_t)w;
  r.hi = (uint32_t)(w >> 32);
  r.base = s - n + (int)(w & 1ull) - 1;
  return r;
}

__device__ __forceinline__ int seg_lookup(const SegIndex& si, int q) {
  const int b = q >> 6, l = q & 63;
  const uint32_t lo = (uint32_t)__shfl((int)si.lo, b), hi = (uint32_t)__shfl((int)si.hi, b);
  const int base = __shfl(si.base, b);
  const unsigned long long w = ((unsigned long long)hi << 32) | lo;
  const unsigned long long upto = (2ull << l) - 1ull;  // bits 0..l (all 64 for l = 63)
  return base + __popcll(w & upto & ~1ull);
}

template <typename T>
__device__ __forceinline__ void weights_from_raw(const DevPlan& P, int pk, uint64_t raw, double& c, double& s) {
  T cc, ss;
  if (pk == 1) {
    const double a = __longlong_as_double((long long)raw);
    if (sizeof(T) == 8) {
      double sd, cd;
      sincos_q(2.0 * a, sd, cd);
      cc = (T)cd;
      ss = (T)sd;
    } else {
      float sf, cf;
      sincos_qf((float)(2.0 * a), sf, cf);
      cc = (T)cf;
      ss = (T)sf;
    }
  } else if (pk == 2) {
    const float a = __uint_as_float((uint32_t)raw);
    if (sizeof(T) == 8) {
      double sd, cd;
      sincos_q(2.0 * (double)a, sd, cd);
      cc = (T)cd;
      ss = (T)sd;
    } else {
      float sf, cf;
      sincos_qf(2.0f * a, sf, cf);
      cc = (T)cf;
      ss = (T)sf;
    }
  } else {
    if (sizeof(T) == 8) {
      const double2 t = P.psi_cs64[(uint32_t)raw];
      cc = (T)t.x;
      ss = (T)t.y;
    } else {
      const float2 t = P.psi_cs32[(uint32_t)raw];
      cc = (T)t.x;
      ss = (T)t.y;
    }
  }
  c = (double)cc;
  s = (double)ss;
}

// LDS layout of k_bin and k_project:
// [stage | acc | carries | start bitmaps (2 x 64 words) | sstart | spos | carry pixels | schunk]
// The stage holds one sub-batch of TOD values (or of P m) in the TOD precision S; acc holds NV
// values for each of the plan's largest tile's tpix pixels; the segment chunks (schunk) are
// only there when the caller needs them (plan pass, d / tau binning).
template <int NV, typename S>
__host__ __device__ constexpr size_t bin_lds_bytes(bool plan, int tpix, bool with_chunk) {
  return (plan ? 0 : kSubBatch * sizeof(S)) + (size_t)tpix * NV * sizeof(double) + kWaves * NV * sizeof(double) +
         2 * (kSubBatch / 64) * sizeof(unsigned long long) + kMaxSegs * (sizeof(int64_t) + sizeof(uint16_t)) +
         kWaves * sizeof(int) + (with_chunk ? kMaxSegs * sizeof(int) : 0);
}

template <typename S>
struct BinLds {
  S* stage;
  double* acc;
  double* cv;
  unsigned long long* smask;  // two bitmaps, alternating between consecutive sub-batches
  int64_t* sstart;
  int* schunk;
  uint16_t* spos;
  int* clp;
};

template <int NV, typename S>
__device__ __forceinline__ BinLds<S> bin_lds(double* base, bool plan, int tpix) {
  BinLds<S> L;
  L.stage = reinterpret_cast<S*>(base);
  L.acc = base + (plan ? 0 : kSubBatch * sizeof(S) / sizeof(double));
  L.cv = L.acc + tpix * NV;
  L.smask = reinterpret_cast<unsigned long long*>(L.cv + kWaves * NV);
  L.sstart = reinterpret_cast<int64_t*>(L.smask + 2 * (kSubBatch / 64));
  L.spos = reinterpret_cast<uint16_t*>(L.sstart + kMaxSegs);
  L.clp = reinterpret_cast<int*>(L.spos + kMaxSegs);
  L.schunk = L.clp + kWaves;
  return L;
}

// Load the segment table of sub-batch S and mark its starts in bitmap `sm` (zeroed beforehand).
// Segment starts are pointing-entry indices: the sample index in time order, plus N_s for the
// second components of composite pointing.  Unless `entries` keeps them (to address the
// two-part projection buffer), they become sample indices; in_work then moves them to the work
// buffer, where chunk c starts at real position 2 xoff_c instead of off_c.  The chunks kept for
// the caller are the samples' chunks.
template <typename SL>
__device__ __forceinline__ void load_segments(const DevPlan& P, const SubBatch& S, const BinLds<SL>& L,
                                              unsigned long long* sm, bool with_chunk, bool in_work,
                                              bool entries = false) {
  const int nseg = S.seg_end - S.seg_begin;
  for (int i = threadIdx.x; i < nseg; i += blockDim.x) {
    const Segment g = P.segs[S.seg_begin + i];
    int64_t start = g.start;
    int chunk = g.chunk;
    if (chunk >= P.nchunk) {
      chunk -= P.nchunk;
      if (!entries) start -= P.nsamp;
    }
    if (in_work) {
      const DevChunk& ch = P.chunks[chunk];
      start += 2 * ch.xoff - ch.off;
    }
    L.sstart[i] = start;
    L.spos[i] = (uint16_t)g.pos;
    if (with_chunk) L.schunk[i] = chunk;
    atomicOr(&sm[g.pos >> 6], 1ull << (g.pos & 63));
  }
}

// kPerLane consecutive entries of a sub-batch's pixel-sorted order, loaded with vector loads:
// local pixels, staging positions and raw angles.  The sorted arrays are padded to kSortAlign
// entries, so a lane whose first entry is in range may read all kPerLane.
struct LaneEntries {
  uint4 lpw[2], pmw[2];
  uint4 psw[kPerLane / 2];  // raw angles: up to 16 x 8 bytes
  uint4 pkw[kPerLane / 4];  // packed entries (stage position, local pixel, angle index)
};

template <bool POL, bool PACKED = false>
__device__ __forceinline__ void load_lane_entries(const DevPlan& P, int pk, int64_t g0, LaneEntries& e) {
  if constexpr (PACKED) {
    const uint4* pp = reinterpret_cast<const uint4*>(P.packed + g0);
#pragma unroll
    for (int w = 0; w < kPerLane / 4; ++w) e.pkw[w] = pp[w];
    return;
  }
  const uint4* lpp = reinterpret_cast<const uint4*>(P.lp + g0);
  const uint4* pmp = reinterpret_cast<const uint4*>(P.perm + g0);
  e.lpw[0] = lpp[0];
  e.lpw[1] = lpp[1];
  e.pmw[0] = pmp[0];
  e.pmw[1] = pmp[1];
  if (POL) {
    const int esz = pk == 1 ? 8 : (pk == 2 ? 4 : 2);
    const int nw = esz;  // uint4 words holding kPerLane angles
    const uint4* pp = reinterpret_cast<const uint4*>((const char*)P.psi_sorted + g0 * esz);
#pragma unroll
    for (int w = 0; w < kPerLane / 2; ++w)
      if (w < nw) e.psw[w] = pp[w];
  }
}

__device__ __forceinline__ int entry_u16(const uint4* w, int i) {
  const uint32_t x = (i < 8) ? ((const uint32_t*)&w[0])[i / 2] : ((const uint32_t*)&w[1])[(i - 8) / 2];
  return (int)((x >> (16 * (i & 1))) & 0xffffu);
}

// entry i of a lane's packed entries: stage position, local pixel, angle index
__device__ __forceinline__ uint32_t entry_packed(const LaneEntries& e, int i) {
  return ((const uint32_t*)e.pkw)[i];
}

__device__ __forceinline__ uint64_t entry_psi_raw(int pk, const LaneEntries& e, int i) {
  const uint32_t* pw = (const uint32_t*)e.psw;
  if (pk == 1) return ((uint64_t)pw[2 * i + 1] << 32) | pw[2 * i];
  if (pk == 2) return pw[i];
  return (pw[i / 2] >> (16 * (i & 1))) & 0xffffu;
}

// P m for every on-map sample of one tile, written to a TOD-sized buffer in time order.
// mt: the tile's map values in LDS, [local pixel][NC].  For each sub-batch, thread q of the
// stage positions reads its sample's local pixel and angle from the plan's stage-order copies,
// forms P m and writes it along the sub-batch's time-contiguous segments (coalesced within each
// segment).  Composite pointing: each component's weighted projection goes to its half of the
// buffer (the segments' entry indices).
template <typename T, int NC, int PK, bool CP>
__device__ void tile_project(const DevPlan& P, const Tile& tl, const double* mt, const BinLds<T>& L, int& sbn,
                             T* __restrict__ pm_out) {
  constexpr int SPW = kSubBatch / kBinBlock;
  // entries in flight per thread: all of them for the FP32 I/Q/U kernels with 16-bit angle
  // indices (their registers allow it), half at a time for the others
  constexpr int kRounds = (NC == 3 && sizeof(T) == 4 && PK == 3) ? 1 : 2, kPer = SPW / kRounds;
  const int pk = PK >= 0 ? PK : P.psi_kind;
  const int esz = pk == 1 ? 8 : (pk == 2 ? 4 : 2);
  for (int sb = tl.sb_begin; sb < tl.sb_end; ++sb, ++sbn) {
    const SubBatch S = P.sbs[sb];
    const int cnt = S.count;
    load_segments(P, S, L, L.smask + (sbn & 1) * (kSubBatch / 64), false, false, true);
    SegIndex si;
#pragma unroll 1
    for (int h = 0; h < kRounds; ++h) {
      // the round's stage entries go out together (the first round's before the segment table
      // is needed)
      int lq[kPer];
      uint64_t rq[kPer];
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int q = threadIdx.x + (h * kPer + u) * kBinBlock;
        const int64_t e = S.sorted_begin + (q < cnt ? q : 0);
        lq[u] = P.lp_stage[e];
        rq[u] = 0;
        if constexpr (NC == 3) {
          const uint8_t* ps = (const uint8_t*)P.psi_stage + e * esz;
          rq[u] = esz == 8 ? *(const uint64_t*)ps : (esz == 4 ? *(const uint32_t*)ps : *(const uint16_t*)ps);
        }
      }
      if (h == 0) {
        __syncthreads();
        si = seg_index(L.smask + (sbn & 1) * (kSubBatch / 64));
        // the other bitmap was last read before the previous sub-batch's final barrier
        if (threadIdx.x < kSubBatch / 64) L.smask[((sbn + 1) & 1) * (kSubBatch / 64) + threadIdx.x] = 0ull;
      }
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int q = threadIdx.x + (h * kPer + u) * kBinBlock;
        const int g = seg_lookup(si, q);  // lane reads with every lane active
        if (q < cnt) {
          const int l = lq[u];
          double v = mt[l * NC];
          if constexpr (NC == 3) {
            double c, sn;
            weights_from_raw<T>(P, pk, rq[u], c, sn);
            v += c * mt[l * 3 + 1] + sn * mt[l * 3 + 2];
          }
          if (CP) v *= q < S.na ? P.wa : P.wb;
          pm_out[L.sstart[g] + (q - (int)L.spos[g])] = (T)v;
        }
      }
    }
    __syncthreads();
  }
}

// PK: the angle kind fixed at compile time (as in the binning kernels; 0 for temperature-only maps)
template <typename T, int NC, int PK, bool CP>
__global__ __launch_bounds__(kBinBlock) void k_project(DevPlan P, const double* __restrict__ m,
                                                       T* __restrict__ pm_out) {
  extern __shared__ double smem_d[];
  const BinLds<T> L = bin_lds<NC, T>(smem_d, false, P.max_tile_pix);
  double* mt = L.acc;
  if (threadIdx.x < 2 * (kSubBatch / 64)) L.smask[threadIdx.x] = 0ull;
  int sbn = 0;
  for (int t = blockIdx.x; t < P.ntiles; t += gridDim.x) {
    const Tile tl = P.tiles[t];
    const int tp = tl.tw * tl.th;
    for (int l = threadIdx.x; l < tp; l += kBinBlock) {
      const int64_t p = (int64_t)(tl.y0 + l / tl.tw) * P.nxm + tl.x0 + (l % tl.tw);
#pragma unroll
      for (int q = 0; q < NC; ++q) mt[l * NC + q] = m[q * P.npix + p];
    }
    __syncthreads();
    tile_project<T, NC, PK, CP>(P, tl, mt, L, sbn, pm_out);
  }
}

// FP32 iteration binning: at most 128 VGPRs, so that four workgroups (36 KB of LDS each) share a CU
// PK: the angle kind fixed at compile time (1 float64, 2 float32, 3 uint16 table index), or -1
// (read from the plan)
// CP: composite pointing (per-entry component weights; compiled out of the single-beam kernels)
template <typename T, int NV, int PK, bool CP>
__global__ __launch_bounds__(kBinBlock, (sizeof(T) == 4 && NV == 3) ? 4 : 1) void k_bin(DevPlan P, int bsrc, const T* __restrict__ src, int epi,
                                                   const double* __restrict__ m_in, double* __restrict__ out,
                                                   double* __restrict__ w_out, int32_t* __restrict__ hits_out,
                                                   uint8_t* __restrict__ sol_out, T* __restrict__ pm_out) {
  constexpr bool PLAN = (NV == 2 || NV == 7);
  constexpr bool POL = (NV == 3 || NV == 7);
  constexpr int SPW = kSubBatch / kBinBlock;  // staged samples per thread
  // the stage holds TOD values in the TOD precision: an FP32 stage cannot hold d / tau exactly
  constexpr bool kScaleAtUse = sizeof(T) < sizeof(double);
  // PK 4: 16-bit table indices, the sorted entries packed (the plan's packed array)
  constexpr bool PACKED = PK == 4;
  const int pk = PACKED ? 3 : (PK >= 0 ? PK : P.psi_kind);
  const int lpb = PACKED ? P.pk_lp_bits : 0;
  const uint32_t lpm = PACKED ? (1u << lpb) - 1u : 0u;
  extern __shared__ double smem_d[];
  const BinLds<T> L = bin_lds<NV, T>(smem_d, PLAN, P.max_tile_pix);
  T* stage = L.stage;
  double* acc = L.acc;
  double* cv = L.cv;
  const int64_t* sstart = L.sstart;
  const uint16_t* spos = L.spos;
  const int* schunk = L.schunk;
  int* clp = L.clp;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x < 2 * (kSubBatch / 64)) L.smask[threadIdx.x] = 0ull;
  int sbn = 0;  // sub-batches processed: selects the start bitmap
  for (int t = blockIdx.x; t < P.ntiles; t += gridDim.x) {
    const Tile tl = P.tiles[t];
    const int tp = tl.tw * tl.th;
    for (int i = threadIdx.x; i < tp * NV; i += kBinBlock) acc[i] = 0.0;
    __syncthreads();
    for (int sb = tl.sb_begin; sb < tl.sb_end; ++sb, ++sbn) {
      const SubBatch S = P.sbs[sb];
      const int cnt = S.count;
      // this wave's stripe of the pixel-sorted order; lane l takes kPerLane consecutive entries
      const int stripe = (((cnt + kWaves - 1) / kWaves) + 63) & ~63;
      const int k0 = wave * stripe;
      const int k1 = min(cnt, k0 + stripe);
      const int kl = k0 + kPerLane * lane;
      const bool active = kl < k1;
      LaneEntries en = {};
      if (active) load_lane_entries<POL, PACKED>(P, pk, S.sorted_begin + kl, en);  // kl: a multiple of kSortAlign
      load_segments(P, S, L, L.smask + (sbn & 1) * (kSubBatch / 64), PLAN || bsrc == BSRC_DATA_OVER_TAU,
                    bsrc == BSRC_WORK);
      if (lane == 0) clp[wave] = -1;
      __syncthreads();
      const SegIndex si = seg_index(L.smask + (sbn & 1) * (kSubBatch / 64));
      // the other bitmap was last read before the previous sub-batch's final barrier
      if (threadIdx.x < kSubBatch / 64) L.smask[((sbn + 1) & 1) * (kSubBatch / 64) + threadIdx.x] = 0ull;
      if (!PLAN) {
        // FP32 I/Q/U: one round of SPW loads in flight per thread; otherwise two rounds of SPW / 2
        constexpr int kRounds = (sizeof(T) == 4 && NV == 3) ? 1 : 2, kPer = SPW / kRounds;
#pragma unroll 1
        for (int h = 0; h < kRounds; ++h) {
          T v[kPer];
#pragma unroll
          for (int u = 0; u < kPer; ++u) {
            const int q = threadIdx.x + (h * kPer + u) * kBinBlock;
            const int gq = seg_lookup(si, q);  // lane reads with every lane active
            if constexpr (sizeof(T) == 4) {
              // FP32: positions past the sub-batch read its first sample (a valid address) and
              // are not stored, so no per-element branch separates the loads (FP64 measured
              // faster with the branch)
              const int g = q < cnt ? gq : 0;
              v[u] = src[sstart[g] + (q < cnt ? q - (int)spos[g] : 0)];
            } else {
              v[u] = 0.0;
              if (q < cnt) {
                v[u] = (double)src[sstart[gq] + (q - (int)spos[gq])];
                // d / tau: scaled here in FP64 staging, where it is used in FP32 staging
                if (bsrc == BSRC_DATA_OVER_TAU) v[u] *= P.chunks[schunk[gq]].inv_tau;
              }
            }
          }
#pragma unroll
          for (int u = 0; u < kPer; ++u) {
            const int q = threadIdx.x + (h * kPer + u) * kBinBlock;
            if (q < cnt) stage[q] = v[u];
          }
        }
        __syncthreads();
      }
      if (k0 < k1) {
        // lane 0 is active
        const int first_lp = __shfl(PACKED ? (int)((en.pkw[0].x >> 12) & lpm) : (int)(en.lpw[0].x & 0xffffu), 0);
        // sequential reduce-by-key over this lane's entries
        int cur_lp = -1, h_lp = -1, nruns = 0;
        double cur[NV], hv[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) cur[q] = hv[q] = 0.0;
#pragma unroll
        for (int i = 0; i < kPerLane; ++i) {
          const int pr = PACKED ? (int)(entry_packed(en, i) & 0xfffu) : entry_u16(en.pmw, i);
          // lane reads with every lane of the wave active
          const int gpr = (PLAN || (kScaleAtUse && bsrc == BSRC_DATA_OVER_TAU)) ? seg_lookup(si, pr) : 0;
          if (kl + i < k1) {
            const int lp = PACKED ? (int)((entry_packed(en, i) >> 12) & lpm) : entry_u16(en.lpw, i);
            double y;
            if (PLAN) {
              y = P.chunks[schunk[gpr]].inv_tau;
            } else {
              y = stage[pr];
              if (kScaleAtUse && bsrc == BSRC_DATA_OVER_TAU) y *= P.chunks[schunk[gpr]].inv_tau;
            }
            if constexpr (CP) {
              // the entry's component weight w; the weight blocks take w^2 / (tau / 2) (T_A = T_B = T/2)
              const double w = pr < S.na ? P.wa : P.wb;
              y *= PLAN ? 2.0 * w * w : w;
            }
            double c = 0.0, sn = 0.0;
            if (POL)
              weights_from_raw<T>(P, pk, PACKED ? (uint64_t)(entry_packed(en, i) >> (12 + lpb)) : entry_psi_raw(pk, en, i),
                                  c, sn);
            double v[NV];
            contrib<T, NV>(P, y, c, sn, v);
            if (lp != cur_lp) {
              if (nruns == 1) {
                h_lp = cur_lp;
#pragma unroll
                for (int q = 0; q < NV; ++q) hv[q] = cur[q];
              } else if (nruns > 1) {
                bin_flush<NV>(acc, cv, clp, wave, cur_lp, first_lp, cur);  // a run inside this lane
              }
              cur_lp = lp;
#pragma unroll
              for (int q = 0; q < NV; ++q) cur[q] = v[q];
              ++nruns;
            } else {
#pragma unroll
              for (int q = 0; q < NV; ++q) cur[q] += v[q];
            }
          }
        }
        // runs that cross lane boundaries: keyed inclusive scan of the lanes' tail runs
        const bool single = nruns <= 1;
        int t_lp = active ? cur_lp : (-2 - lane);
        if (single) h_lp = t_lp;
        double Sv[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) Sv[q] = active ? cur[q] : 0.0;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
          const int uk = __shfl_up(t_lp, dd);
          double us[NV];
#pragma unroll
          for (int q = 0; q < NV; ++q) us[q] = __shfl_up(Sv[q], dd);
          if (lane >= dd && uk == t_lp) {
#pragma unroll
            for (int q = 0; q < NV; ++q) Sv[q] += us[q];
          }
        }
        int prev_key = __shfl_up(t_lp, 1);
        double prev_S[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) prev_S[q] = __shfl_up(Sv[q], 1);
        int next_h = __shfl_down(h_lp, 1);
        if (lane == 0) prev_key = -1;
        if (lane == 63) next_h = -1;
        // a lane with several runs completes its head run (adding what earlier lanes carried in)
        if (active && !single) {
          if (h_lp == prev_key) {
#pragma unroll
            for (int q = 0; q < NV; ++q) hv[q] += prev_S[q];
          }
          bin_flush<NV>(acc, cv, clp, wave, h_lp, first_lp, hv);
        }
        // the tail run ends here unless the next lane continues it
        if (active && next_h != t_lp) bin_flush<NV>(acc, cv, clp, wave, t_lp, first_lp, Sv);
      }
      __syncthreads();
      if (threadIdx.x < NV) {
        for (int w = 0; w < kWaves; ++w) {
          const int l = clp[w];
          if (l >= 0) acc[l * NV + threadIdx.x] += cv[w * NV + threadIdx.x];
        }
      }
      __syncthreads();
    }
    // epilogue: one thread per pixel of the tile
    for (int l = threadIdx.x; l < tp; l += kBinBlock) {
      const int64_t p = (int64_t)(tl.y0 + l / tl.tw) * P.nxm + tl.x0 + (l % tl.tw);
      const double* a = acc + l * NV;
      if (epi == EPI_PLAN) {
        const double hits = a[0];
        hits_out[p] = (int32_t)hits;
        bool ok = hits > 0.5;
        if (NV == 2) {
          ok = ok && a[1] > 0.0;
          w_out[p] = ok ? 1.0 / a[1] : 0.0;
        } else {
          const double w00 = a[1], w01 = a[2], w02 = a[3], w11 = a[4], w12 = a[5], w22 = a[6];
          const double c00 = w11 * w22 - w12 * w12;
          const double c01 = w02 * w12 - w01 * w22;
          const double c02 = w01 * w12 - w02 * w11;
          const double c11 = w00 * w22 - w02 * w02;
          const double c12 = w01 * w02 - w00 * w12;
          const double c22 = w00 * w11 - w01 * w01;
          const double det = w00 * c00 + w01 * c01 + w02 * c02;
          double i00 = 0, i01 = 0, i02 = 0, i11 = 0, i12 = 0, i22 = 0;
          // solvable: hits and det(W) / (W00 W11 W22) >= 1e-8 (angle coverage separates Q and U)
          const double diag = w00 * w11 * w22;
          ok = ok && diag > 0.0 && det >= 1e-8 * diag;
          if (ok) {
            const double id = 1.0 / det;
            i00 = c00 * id;
            i01 = c01 * id;
            i02 = c02 * id;
            i11 = c11 * id;
            i12 = c12 * id;
            i22 = c22 * id;
          }
          if (!ok) i00 = i01 = i02 = i11 = i12 = i22 = 0.0;
          const int64_t np = P.npix;
          w_out[p] = i00;
          w_out[np + p] = i01;
          w_out[2 * np + p] = i02;
          w_out[3 * np + p] = i11;
          w_out[4 * np + p] = i12;
          w_out[5 * np + p] = i22;
        }
        sol_out[p] = ok ? 1 : 0;
      } else if (epi == EPI_WRITE_B) {
#pragma unroll
        for (int q = 0; q < NV; ++q) out[q * P.npix + p] = a[q];
      } else {
        const bool ok = P.solvable[p] != 0;
        const int64_t np = P.npix;
        double u[NV > 3 ? NV : 3];
        if (NV == 1) {
          u[0] = P.winv[p] * a[0];
        } else if (NV == 3) {
          const double i00 = P.winv[p], i01 = P.winv[np + p], i02 = P.winv[2 * np + p];
          const double i11 = P.winv[3 * np + p], i12 = P.winv[4 * np + p], i22 = P.winv[5 * np + p];
          u[0] = i00 * a[0] + i01 * a[1] + i02 * a[2];
          u[1] = i01 * a[0] + i11 * a[1] + i12 * a[2];
          u[2] = i02 * a[0] + i12 * a[1] + i22 * a[2];
        }
        double rr[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          double r = 0.0;
          if (ok)
            r = (epi == EPI_UPDATE)     ? m_in[q * np + p] + u[q]
                : (epi == EPI_MAPSIZED) ? P.md[q * np + p] + m_in[q * np + p] - u[q]
                                        : u[q];
          out[q * np + p] = r;
          rr[q] = r;
          if (!PLAN && pm_out) acc[l * NV + q] = r;  // the tile's new map values, for P m below
        }
        if (NV == 3 && P.mapi && (epi == EPI_UPDATE || epi == EPI_REPLACE || epi == EPI_MAPSIZED)) {
          P.mapi[2 * p] = make_double2(rr[0], rr[NV > 1 ? 1 : 0]);
          P.mapi[2 * p + 1] = make_double2(rr[NV > 2 ? 2 : 0], 0.0);
        }
      }
    }
    __syncthreads();
    if (!PLAN && pm_out && (epi == EPI_UPDATE || epi == EPI_REPLACE || epi == EPI_MAPSIZED))
      tile_project<T, (NV == 3 ? 3 : 1), (PACKED ? 3 : PK), CP>(P, tl, acc, L, sbn, pm_out);
  }
}

// ---------------------------------------------------------------------------------------------
// gradient of the solved map with respect to each chunk's noise parameters
//
// With r = d - P m (m the GLS map) and z = A^-1 g (the adjoint map of a loss gradient g),
// dL/dtheta_c = -(1/n_c) sum_k omega_k Re(conj(Zhat_k) Rhat_k) (dN_k/dtheta_c) / N_k^2 over the
// real bins of chunk c, Zhat = rfft of P z.  Both residuals arrive in their column-transformed
// row layout (pass A output); the row transforms and the real-spectrum untangle are those of
// pass B.  theta = (sigma, fknee, alpha): dN/dsigma = 2 N / sigma, dN/dfknee = -alpha pl / fknee,
// dN/dalpha = pl ln(f / fknee), pl = sigma^2 (f/fknee)^alpha (f_0 -> f_1).

template <typename T>
__device__ __forceinline__ void grad_bin(const DevPlan& P, const DevChunk& ch, int k, double w, cx<T> R, cx<T> Z,
                                         double* acc) {
  const double pl = (double)powerlaw_bin<T>(P, ch, k, spec_index(ch, k));
  const double N = ch.sigma2 + pl;
  const double f = (double)(k == 0 ? 1 : k) * ch.df;
  const double cross = (double)Z.x * (double)R.x + (double)Z.y * (double)R.y;
  const double c = -w * cross / ((double)ch.n * N * N);
  acc[0] += c * 2.0 * N / sqrt(ch.sigma2);
  acc[1] += c * (-ch.alpha * pl / ch.fknee);
  acc[2] += c * pl * log(f / ch.fknee);
}

template <typename T>
__device__ __forceinline__ void untangle(const DevClass& cl, const DevPlan& P, cx<T> Zk, cx<T> Zm, int k, cx<T>& Rk,
                                         cx<T>& Rm) {
  cx<T> E, O;
  E.x = T(0.5) * (Zk.x + Zm.x);
  E.y = T(0.5) * (Zk.y - Zm.y);
  O.x = T(0.5) * (Zk.y + Zm.y);
  O.y = -T(0.5) * (Zk.x - Zm.x);
  const cx<T> wO = cmul(omega2M<T>(P, cl, k), O);
  Rk = cadd(E, wO);
  Rm = csub(conjc(E), conjc(wO));
}

template <typename T>
__global__ __launch_bounds__(kBlockB) void k_grad_b(DevPlan P, const ItemB* __restrict__ items, int nitems,
                                                   const cx<T>* __restrict__ Xr, const cx<T>* __restrict__ Xz,
                                                   double* __restrict__ part) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const ItemB item = items[it];
    const DevChunk ch = P.chunks[item.chunk];
    const DevClass& cl = P.classes[ch.cls];
    const int M1 = ch.M1, M2 = ch.M2, M = ch.M;
    const int ra = item.ra, rb = item.rb;
    const int nrow = (ra == rb) ? 1 : 2;
    // sequences: rows of r at [0, nrow*M1), rows of P z at [nrow*M1, 2*nrow*M1)
    const int off2 = nrow * M1;
    for (int e = threadIdx.x; e < M1; e += kBlockB) {
      lds[e] = Xr[ch.xoff + (int64_t)ra * M1 + e];
      lds[off2 + e] = Xz[ch.xoff + (int64_t)ra * M1 + e];
      if (nrow == 2) {
        lds[M1 + e] = Xr[ch.xoff + (int64_t)rb * M1 + e];
        lds[off2 + M1 + e] = Xz[ch.xoff + (int64_t)rb * M1 + e];
      }
    }
    __syncthreads();
    // the rows of r, then those of P z: each call holds at most the row pass's two rows, within
    // the NT * Ept values a transform call covers
    lds_fft<T, false, false, kBlockB>(lds, M1, nrow, 0, cl.rad1, cl.nr1, twtab<T>(P) + cl.tw1);
    lds_fft<T, false, false, kBlockB>(lds + off2, M1, nrow, 0, cl.rad1, cl.nr1, twtab<T>(P) + cl.tw1);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int sl = 0; sl < nrow; ++sl) {
      const int row = sl == 0 ? ra : rb;
      const bool self = (row == 0) || (2 * row == M2);
      if (!self && sl == 1) break;  // a row pair is handled from its first row
      for (int k1 = threadIdx.x; k1 < M1; k1 += kBlockB) {
        int prow, pk1;
        if (!self) {
          prow = 1;
          pk1 = M1 - 1 - k1;
        } else {
          prow = sl;
          pk1 = (row == 0) ? (k1 == 0 ? 0 : M1 - k1) : (M1 - 1 - k1);
          if (k1 > pk1) continue;
        }
        const int k = row + M2 * k1;
        const int ia = sl * M1 + k1, ib = prow * M1 + pk1;
        const cx<T> Ra = lds[ia], Rb = lds[ib], Za = lds[off2 + ia], Zb = lds[off2 + ib];
        if (k == 0) {
          cx<T> R0, RM, Z0, ZM;
          R0.x = Ra.x + Ra.y;
          R0.y = T(0);
          RM.x = Ra.x - Ra.y;
          RM.y = T(0);
          Z0.x = Za.x + Za.y;
          Z0.y = T(0);
          ZM.x = Za.x - Za.y;
          ZM.y = T(0);
          grad_bin<T>(P, ch, 0, 1.0, R0, Z0, acc);
          grad_bin<T>(P, ch, M, 1.0, RM, ZM, acc);
        } else if (ia == ib) {
          grad_bin<T>(P, ch, k, 2.0, conjc(Ra), conjc(Za), acc);
        } else {
          cx<T> Rk, Rm, Zk, Zm;
          untangle<T>(cl, P, Ra, Rb, k, Rk, Rm);
          untangle<T>(cl, P, Za, Zb, k, Zk, Zm);
          grad_bin<T>(P, ch, k, 2.0, Rk, Zk, acc);
          grad_bin<T>(P, ch, M - k, 2.0, Rm, Zm, acc);
        }
      }
    }
    __syncthreads();  // the spectra are no longer needed: reuse the LDS for the reduction
    double* red = reinterpret_cast<double*>(smem_raw);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double v = acc[q];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if ((threadIdx.x & 63) == 0) red[q * (kBlockB / 64) + (threadIdx.x >> 6)] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
      double t = 0.0;
      for (int w = 0; w < kBlockB / 64; ++w) t += red[threadIdx.x * (kBlockB / 64) + w];
      part[3 * (int64_t)it + threadIdx.x] = t;
    }
    __syncthreads();
  }
}

// per-chunk sums of the (nitems x 3) partials in item order
__global__ __launch_bounds__(kBlock) void k_grad_reduce(const int32_t* __restrict__ chunk_item_begin,
                                                        const double* __restrict__ part, int nchunk,
                                                        double* __restrict__ out) {
  __shared__ double red[kBlock];
  const int c = blockIdx.x;
  for (int q = 0; q < 3; ++q) {
    double s = 0.0;
    for (int i = chunk_item_begin[c] + threadIdx.x; i < chunk_item_begin[c + 1]; i += kBlock) s += part[3 * i + q];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[3 * c + q] = red[0];
    __syncthreads();
  }
}

hipError_t launch_grad(const DevPlan& P, const ItemB* items, int nitems, const int32_t* chunk_item_begin,
                       const void* Xr, const void* Xz, double* part, double* out, size_t lds, hipStream_t s) {
  const size_t tot = lds > 3 * (kBlockB / 64) * sizeof(double) ? lds : 3 * (kBlockB / 64) * sizeof(double);
  if (P.precision == 0)
    hipLaunchKernelGGL(k_grad_b<double>, dim3(grid_for(nitems, kGridCap)), dim3(kBlockB), tot, s, P, items, nitems,
                       (const double2*)Xr, (const double2*)Xz, part);
  else
    hipLaunchKernelGGL(k_grad_b<float>, dim3(grid_for(nitems, kGridCap)), dim3(kBlockB), tot, s, P, items, nitems,
                       (const float2*)Xr, (const float2*)Xz, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_reduce, dim3(P.nchunk), dim3(kBlock), 0, s, chunk_item_begin, part, P.nchunk, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// chi^2 per Fourier mode, summed in log-spaced bins (a diagnostic of the noise model)
//
// Real bin k of a chunk falls in bin 0 for k = 0 and otherwise, with o = floor(log2 k) and s bins
// per octave, in bin 1 + s o + floor(s (k - 2^o) / 2^o).  Bin b >= 1 therefore holds
// k - 2^o in [ceil(j 2^o / s), ceil((j + 1) 2^o / s)) with o = (b - 1) / s, j = (b - 1) mod s.
// One workgroup per (listed chunk, bin): the chunk's terms in that range summed in a fixed order,
// and the number of real modes they stand for (2 per bin, 1 for k = 0 and k = n/2).

__global__ __launch_bounds__(256) void k_modes_bin(const double* __restrict__ modes, int64_t M, int per_octave,
                                                   double* __restrict__ out) {
  __shared__ double red[256];
  const int b = blockIdx.x;  // the chunk's terms cover k = 0 .. M
  int64_t lo, hi;
  if (b == 0) {
    lo = 0;
    hi = 1;
  } else {
    const int o = (b - 1) / per_octave, j = (b - 1) % per_octave;
    const int64_t p2 = (int64_t)1 << o;
    lo = p2 + (j * p2 + per_octave - 1) / per_octave;
    hi = p2 + ((j + 1) * p2 + per_octave - 1) / per_octave;
  }
  if (hi > M + 1) hi = M + 1;
  double sacc = 0.0;
  for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) sacc += modes[k];
  red[threadIdx.x] = sacc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double cnt = 0.0;
    if (hi > lo) {
      cnt = 2.0 * (double)(hi - lo);
      if (lo == 0) cnt -= 1.0;
      if (hi == M + 1) cnt -= 1.0;
    }
    out[2 * b] = red[0];
    out[2 * b + 1] = cnt;
  }
}

hipError_t launch_modes_bin(const double* modes, int64_t M, int per_octave, int nbins, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_modes_bin, dim3(nbins), dim3(256), 0, s, modes, M, per_octave, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// plan: tabulate the power-law part of every chunk's noise spectrum (FP64 form)

__global__ void k_spectrum(DevPlan P, double* __restrict__ spec) {
  const int c = blockIdx.y;
  const DevChunk ch = P.chunks[c];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= ch.M; i += gridDim.x * blockDim.x) {
    const int k = (i == ch.M) ? ch.M : (i % ch.M1) * ch.M2 + i / ch.M1;  // inverse of the row layout
    spec[ch.spec_off + i] = powerlaw<double>(ch, k);
  }
}

hipError_t launch_spectrum(const DevPlan& P, double* spec, hipStream_t s) {
  hipLaunchKernelGGL(k_spectrum, dim3(64, P.nchunk), dim3(256), 0, s, P, spec);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// reductions and map-space vector kernels (all deterministic: fixed partition, fixed tree)

__global__ __launch_bounds__(kBlock) void k_chi2_reduce(const int32_t* __restrict__ chunk_item_begin,
                                                        const double* __restrict__ part, int nchunk,
                                                        double* __restrict__ per_chunk, double* __restrict__ total) {
  __shared__ double red[kBlock];
  // one workgroup: chunk sums in chunk order, then the total
  double acc_total = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    double s = 0.0;
    for (int i = chunk_item_begin[c] + threadIdx.x; i < chunk_item_begin[c + 1]; i += kBlock) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      if (per_chunk) per_chunk[c] = red[0];
      acc_total += red[0];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = acc_total;
}

__global__ void k_fill(double* x, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}
__global__ void k_copy(double* dst, const double* src, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
__global__ void k_copy_bytes(uint8_t* dst, const uint8_t* src, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
__global__ void k_sub(double* out, const double* a, const double* b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = a[i] - b[i];
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kBlock) void k_dot_partials(const double* __restrict__ a, const double* __restrict__ b,
                                                         int64_t n, double* __restrict__ part) {
  __shared__ double red[kBlock];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    s += a[i] * b[i];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_reduce(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double red[kBlock];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) s += part[i];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) *out = t;
}

__device__ __forceinline__ void winv_apply_one(const DevPlan& P, int64_t p, const double* x, double* y) {
  const int64_t np = P.npix;
  if (P.ncomp == 1) {
    y[p] = P.winv[p] * x[p];
    return;
  }
  const double a0 = x[p], a1 = x[np + p], a2 = x[2 * np + p];
  const double i00 = P.winv[p], i01 = P.winv[np + p], i02 = P.winv[2 * np + p];
  const double i11 = P.winv[3 * np + p], i12 = P.winv[4 * np + p], i22 = P.winv[5 * np + p];
  y[p] = i00 * a0 + i01 * a1 + i02 * a2;
  y[np + p] = i01 * a0 + i11 * a1 + i12 * a2;
  y[2 * np + p] = i02 * a0 + i12 * a1 + i22 * a2;
}

__global__ void k_winv_apply(DevPlan P, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P.npix; p += (int64_t)gridDim.x * blockDim.x)
    winv_apply_one(P, p, x, y);
}

// x += alpha p, r -= alpha q, z = W^-1 r, partial sums of r.z ; alpha = rz / pq
__global__ __launch_bounds__(kBlock) void k_cg_update_xr(DevPlan P, double* __restrict__ x, double* __restrict__ r,
                                                         double* __restrict__ z, const double* __restrict__ p,
                                                         const double* __restrict__ q, const double* __restrict__ rz,
                                                         const double* __restrict__ pq, double* __restrict__ part) {
  __shared__ double red[kBlock];
  const double alpha = (*rz) / (*pq);
  const int64_t np = P.npix;
  const int nc = P.ncomp;
  double s = 0.0;
  for (int64_t pix = blockIdx.x * (int64_t)kBlock + threadIdx.x; pix < np; pix += (int64_t)gridDim.x * kBlock) {
    for (int c = 0; c < nc; ++c) {
      const int64_t i = c * np + pix;
      x[i] += alpha * p[i];
      r[i] -= alpha * q[i];
    }
    winv_apply_one(P, pix, r, z);
    for (int c = 0; c < nc; ++c) s += r[c * np + pix] * z[c * np + pix];
  }
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// p = z + (rz_new / rz_old) p
__global__ void k_cg_update_p(double* __restrict__ p, const double* __restrict__ z, const double* __restrict__ rz_new,
                              const double* __restrict__ rz_old, int64_t n) {
  const double beta = (*rz_new) / (*rz_old);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = z[i] + beta * p[i];
}

__global__ void k_cg_chi2(const double* chi2_0, const double* xb, const double* xr, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = *chi2_0 - *xb - *xr;
}

// ---------------------------------------------------------------------------------------------
// launchers


template <typename T, bool P2>
static void launch_pass_a_t(const DevPlan& P, const ItemAC* items, int nitems, const void* d, const double* m,
                            int src, void* work, size_t lds, hipStream_t s, const void* pmbuf) {
  const bool ng = src == SRC_D || src == SRC_PMBUF || src == SRC_D_MINUS_PMBUF || src == SRC_GAP;
  // a second stream: gap filling's d_0, or the P_B m half of a composite plan's projection buffer
  const bool x2 = src == SRC_GAP || (P.pmb_off != 0 && (src == SRC_PMBUF || src == SRC_D_MINUS_PMBUF));
#define MM_PASS_A(NGV, PKV, X2V)                                                                          \
  hipLaunchKernelGGL((k_pass_a<T, P2, NGV, PKV, X2V>), dim3(col_grid(nitems)), dim3(kBlock), lds, s, P, items, \
                     nitems, (const T*)d, m, src, (cx<T>*)work, (const T*)pmbuf)
  if (ng && x2) {
    MM_PASS_A(true, -1, true);
  } else if (ng) {
    MM_PASS_A(true, -1, false);
  } else {
    switch (P.ncomp == 1 ? 0 : P.psi_kind) {
      case 0: MM_PASS_A(false, 0, false); break;
      case 1: MM_PASS_A(false, 1, false); break;
      case 2: MM_PASS_A(false, 2, false); break;
      default: MM_PASS_A(false, 3, false); break;
    }
  }
#undef MM_PASS_A
}

hipError_t launch_pass_a(const DevPlan& P, const ItemAC* items, int nitems, const void* d, const double* m, int src,
                         void* work, size_t lds, hipStream_t s, const void* pmbuf) {
  if (nitems <= 0) return hipSuccess;
  // the inlined power-of-two transforms fit the FP64 tiles; the FP32 tiles (16 values per
  // thread) spill with them, so FP32 keeps the out-of-line stages
  const bool p2 = P.all_pow2 != 0 && P.precision == 0;
  if (P.precision == 0) {
    if (p2)
      launch_pass_a_t<double, true>(P, items, nitems, d, m, src, work, lds, s, pmbuf);
    else
      launch_pass_a_t<double, false>(P, items, nitems, d, m, src, work, lds, s, pmbuf);
  } else {
    launch_pass_a_t<float, false>(P, items, nitems, d, m, src, work, lds, s, pmbuf);
  }
  return hipGetLastError();
}

hipError_t launch_pass_b(const DevPlan& P, const ItemB* items, int nitems, void* work, int ops, int gain, double lam,
                         double chi2_lam, double* chi2_part, size_t lds, hipStream_t s, double* modes) {
  if (nitems <= 0) return hipSuccess;
  BinCtx bc;
  bc.gain = gain;
  bc.chi2 = (ops & B_CHI2) ? 1 : 0;
  bc.modes = modes;
  bc.lam = lam;
  bc.inv_lam = 1.0 / lam;
  bc.chi2_lam = chi2_lam;
  const int red_off = (int)lds;
  const size_t tot = lds + (kBlockB / 64) * sizeof(double);
  // the row pass keeps the out-of-line stages: inlined, its 128-VGPR bound made it spill
  if (P.precision == 0)
    hipLaunchKernelGGL(k_pass_b<double>, dim3(grid_for(nitems, kGridCap)), dim3(kBlockB), tot, s, P, items,
                       nitems, (double2*)work, ops, bc, chi2_part, red_off);
  else
    hipLaunchKernelGGL(k_pass_b<float>, dim3(grid_for(nitems, kGridCap)), dim3(kBlockB), tot, s, P, items,
                       nitems, (float2*)work, ops, bc, chi2_part, red_off);
  return hipGetLastError();
}

template <typename T, bool P2>
static void launch_pass_c_t(const DevPlan& P, const ItemAC* items, int nitems, void* work, size_t lds, hipStream_t s) {
  const dim3 g(col_grid(nitems)), b(kBlock);
  if (P2 || P.col_wave == 0)
    hipLaunchKernelGGL((k_pass_c<T, P2, 0>), g, b, lds, s, P, items, nitems, (cx<T>*)work);
  else if (P.col_wave == 3 && sizeof(T) == 4)
    hipLaunchKernelGGL((k_pass_c<float, false, 3>), g, b, lds, s, P, items, nitems, (float2*)work);
  else if (P.col_wave == 1)
    hipLaunchKernelGGL((k_pass_c<T, false, 1>), g, b, lds, s, P, items, nitems, (cx<T>*)work);
  else
    hipLaunchKernelGGL((k_pass_c<T, false, 2>), g, b, lds, s, P, items, nitems, (cx<T>*)work);
}

hipError_t launch_pass_c(const DevPlan& P, const ItemAC* items, int nitems, void* work, size_t lds, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  // FP64 power-of-two plans: inlined workgroup-wide stages (the plan then selects no wave-local
  // class); otherwise the layouts the plan selected, with out-of-line stages
  const bool p2 = P.all_pow2 != 0 && P.precision == 0;
  if (P.precision == 0) {
    if (p2)
      launch_pass_c_t<double, true>(P, items, nitems, work, lds, s);
    else
      launch_pass_c_t<double, false>(P, items, nitems, work, lds, s);
  } else {
    launch_pass_c_t<float, false>(P, items, nitems, work, lds, s);
  }
  return hipGetLastError();
}

template <typename T, int NV>
static hipError_t launch_bin_t(const DevPlan& P, int bsrc, const void* src, int epi, const double* m_in, double* out,
                               double* w_out, int32_t* hits_out, uint8_t* sol_out, hipStream_t s, void* pm_out) {
  constexpr bool plan = NV == 2 || NV == 7;
  const size_t lds = bin_lds_bytes<NV, T>(plan, P.max_tile_pix, plan || bsrc == BSRC_DATA_OVER_TAU);
#define MM_BIN_CP(PKV, CPV)                                                                              \
  hipLaunchKernelGGL((k_bin<T, NV, PKV, CPV>), dim3(grid_for(P.ntiles, kGridCap)), dim3(kBinBlock), lds, s, P, \
                     bsrc, (const T*)src, epi, m_in, out, w_out, hits_out, sol_out, (T*)pm_out)
#define MM_BIN(PKV)             \
  if (P.composite)              \
    MM_BIN_CP(PKV, true);       \
  else                          \
    MM_BIN_CP(PKV, false)
  // the I/Q/U iteration kernels take the angle kind at compile time; packed sorted entries (I/Q/U
  // plans with 16-bit angle indices that fit) take the packed variant, the plan pass's too
  if constexpr (NV == 3 || NV == 7) {
    if (P.packed) {
      MM_BIN(4);
      return hipGetLastError();
    }
  }
  if constexpr (NV != 3) {
    MM_BIN(-1);
  } else {
    switch (P.psi_kind) {
      case 1: MM_BIN(1); break;
      case 2: MM_BIN(2); break;
      default: MM_BIN(3); break;
    }
  }
#undef MM_BIN
#undef MM_BIN_CP
  return hipGetLastError();
}

__global__ void k_interleave(DevPlan P, const double* __restrict__ m) {
  const int64_t np = P.npix;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
    P.mapi[2 * p] = make_double2(m[p], m[np + p]);
    P.mapi[2 * p + 1] = make_double2(m[2 * np + p], 0.0);
  }
}

template <typename T>
__global__ void k_unshift(DevPlan P, const T* __restrict__ work, T* __restrict__ out) {
  for (int c = blockIdx.x; c < P.nchunk; c += gridDim.x) {
    const DevChunk& ch = P.chunks[c];
    const T* src = work + 2 * ch.xoff;
    T* dst = out + ch.off;
    for (int t = threadIdx.x; t < ch.n; t += blockDim.x) dst[t] = src[t];
  }
}

// gap filling, time-domain steps (one workgroup per chunk at a time, like k_unshift)
template <typename T>
__global__ void k_gap_init(DevPlan P, const T* __restrict__ d, const uint8_t* __restrict__ gaps, T* __restrict__ d0,
                           T* __restrict__ t0) {
  for (int c = blockIdx.x; c < P.nchunk; c += gridDim.x) {
    const DevChunk& ch = P.chunks[c];
    for (int t = threadIdx.x; t < ch.n; t += blockDim.x) {
      const int64_t j = ch.off + t;
      const T v = gaps[j] ? T(0) : d[j];
      d0[j] = v;
      t0[j] = v;
    }
  }
}

// d_0 = t_1 + y, t_1 = d outside the gaps and d_0 inside (y: the filtered t_0 - t_1)
template <typename T>
__global__ void k_gap_d0(DevPlan P, const T* __restrict__ d, const uint8_t* __restrict__ gaps,
                         const T* __restrict__ work, T* __restrict__ d0) {
  for (int c = blockIdx.x; c < P.nchunk; c += gridDim.x) {
    const DevChunk& ch = P.chunks[c];
    const T* y = work + 2 * ch.xoff;
    for (int t = threadIdx.x; t < ch.n; t += blockDim.x) {
      const int64_t j = ch.off + t;
      const double t1 = gaps[j] ? (double)d0[j] : (double)d[j];
      d0[j] = (T)(t1 + (double)y[t]);
    }
  }
}

// t_0 = P m + tau y (y: the messenger-filtered d_0 - P m)
template <typename T>
__global__ void k_gap_t0(DevPlan P, const T* __restrict__ pm, const T* __restrict__ work, T* __restrict__ t0) {
  for (int c = blockIdx.x; c < P.nchunk; c += gridDim.x) {
    const DevChunk& ch = P.chunks[c];
    const T* y = work + 2 * ch.xoff;
    const double tau = ch.tau;
    for (int t = threadIdx.x; t < ch.n; t += blockDim.x) {
      const int64_t j = ch.off + t;
      t0[j] = (T)((double)pm[j] + tau * (double)y[t]);
    }
  }
}

hipError_t launch_gap_init(const DevPlan& P, const void* d, const uint8_t* gaps, void* d0, void* t0, hipStream_t s) {
  const int g = P.nchunk < 65536 ? P.nchunk : 65536;
  if (P.precision == 0)
    hipLaunchKernelGGL(k_gap_init<double>, dim3(g), dim3(256), 0, s, P, (const double*)d, gaps, (double*)d0,
                       (double*)t0);
  else
    hipLaunchKernelGGL(k_gap_init<float>, dim3(g), dim3(256), 0, s, P, (const float*)d, gaps, (float*)d0,
                       (float*)t0);
  return hipGetLastError();
}

hipError_t launch_gap_d0(const DevPlan& P, const void* d, const uint8_t* gaps, const void* work, void* d0,
                         hipStream_t s) {
  const int g = P.nchunk < 65536 ? P.nchunk : 65536;
  if (P.precision == 0)
    hipLaunchKernelGGL(k_gap_d0<double>, dim3(g), dim3(256), 0, s, P, (const double*)d, gaps, (const double*)work,
                       (double*)d0);
  else
    hipLaunchKernelGGL(k_gap_d0<float>, dim3(g), dim3(256), 0, s, P, (const float*)d, gaps, (const float*)work,
                       (float*)d0);
  return hipGetLastError();
}

hipError_t launch_gap_t0(const DevPlan& P, const void* pm, const void* work, void* t0, hipStream_t s) {
  const int g = P.nchunk < 65536 ? P.nchunk : 65536;
  if (P.precision == 0)
    hipLaunchKernelGGL(k_gap_t0<double>, dim3(g), dim3(256), 0, s, P, (const double*)pm, (const double*)work,
                       (double*)t0);
  else
    hipLaunchKernelGGL(k_gap_t0<float>, dim3(g), dim3(256), 0, s, P, (const float*)pm, (const float*)work,
                       (float*)t0);
  return hipGetLastError();
}

hipError_t launch_unshift(const DevPlan& P, const void* work, void* out, hipStream_t s) {
  const int g = P.nchunk < 65536 ? P.nchunk : 65536;
  if (P.precision == 0)
    hipLaunchKernelGGL(k_unshift<double>, dim3(g), dim3(256), 0, s, P, (const double*)work, (double*)out);
  else
    hipLaunchKernelGGL(k_unshift<float>, dim3(g), dim3(256), 0, s, P, (const float*)work, (float*)out);
  return hipGetLastError();
}

// Binning by global FP64 atomics, the measured alternative to the sorted segmented reduction:
// samples in time order (coalesced reads of y, pix and the angles), one atomic add per map
// component per on-map sample.  The order of the additions, hence the rounding, varies from run
// to run.  Block (x, c) covers samples [x * 4096, (x + 1) * 4096) of chunk c.
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_bin_atomic(DevPlan P, int bsrc, const T* __restrict__ src,
                                                    double* __restrict__ b) {
  const int np = (int)P.npix;
  for (int c = blockIdx.y; c < P.nchunk; c += gridDim.y) {
    const DevChunk& ch = P.chunks[c];
    // y of the work buffer sits at 2 xoff + (t - off); the data are in time order
    const T* sc = src + (bsrc == BSRC_WORK ? 2 * ch.xoff : ch.off);
    const double scale = bsrc == BSRC_WORK ? 1.0 : ch.inv_tau;
    for (int t0 = blockIdx.x * 4096; t0 < ch.n; t0 += gridDim.x * 4096) {
      const int t1 = min(ch.n, t0 + 4096);
      for (int t = t0 + (int)threadIdx.x; t < t1; t += 256) {
        const int64_t j = ch.off + t;
        const int p = P.pix[j];
        if (p < 0) continue;
        const double y = (double)sc[t] * scale;
        unsafeAtomicAdd(&b[p], y);
        if (NC == 3) {
          T cc, ss;
          psi_weights<T>(P, P.psi, j, cc, ss);
          unsafeAtomicAdd(&b[np + p], (double)cc * y);
          unsafeAtomicAdd(&b[2 * np + p], (double)ss * y);
        }
      }
    }
  }
}

// The binning epilogue's per-pixel step from a binned vector b: m_out = m_in + W^-1 b (EPI_UPDATE),
// W^-1 b (EPI_REPLACE) or m_d + m_in - W^-1 b (EPI_MAPSIZED) on solvable pixels, 0 elsewhere;
// refreshes the interleaved map.
template <int NC>
__global__ __launch_bounds__(256) void k_update(DevPlan P, int epi, const double* __restrict__ m_in,
                                                const double* __restrict__ b, double* __restrict__ out) {
  const int64_t np = P.npix;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
    const bool ok = P.solvable[p] != 0;
    double u[3];
    if (NC == 1) {
      u[0] = P.winv[p] * b[p];
    } else {
      const double a0 = b[p], a1 = b[np + p], a2 = b[2 * np + p];
      const double i00 = P.winv[p], i01 = P.winv[np + p], i02 = P.winv[2 * np + p];
      const double i11 = P.winv[3 * np + p], i12 = P.winv[4 * np + p], i22 = P.winv[5 * np + p];
      u[0] = i00 * a0 + i01 * a1 + i02 * a2;
      u[1] = i01 * a0 + i11 * a1 + i12 * a2;
      u[2] = i02 * a0 + i12 * a1 + i22 * a2;
    }
    double r[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      if (ok)
        r[q] = (epi == EPI_UPDATE)     ? m_in[q * np + p] + u[q]
               : (epi == EPI_MAPSIZED) ? P.md[q * np + p] + m_in[q * np + p] - u[q]
                                       : u[q];
      out[q * np + p] = r[q];
    }
    if (NC == 3 && P.mapi) {
      P.mapi[2 * p] = make_double2(r[0], r[1]);
      P.mapi[2 * p + 1] = make_double2(r[2], 0.0);
    }
  }
}

hipError_t launch_bin_atomic(const DevPlan& P, int bsrc, const void* src, double* b, int64_t max_n, hipStream_t s) {
  // the longest chunk sets the x extent (blocks past a shorter chunk's end exit at once)
  const int gx = (int)std::min<int64_t>((max_n + 4095) / 4096, 1024);
  const int gy = P.nchunk < 65535 ? P.nchunk : 65535;
  const dim3 grid(gx < 1 ? 1 : gx, gy);
  const bool f64 = P.precision == 0;
  if (P.ncomp == 1) {
    if (f64)
      hipLaunchKernelGGL((k_bin_atomic<double, 1>), grid, dim3(256), 0, s, P, bsrc, (const double*)src, b);
    else
      hipLaunchKernelGGL((k_bin_atomic<float, 1>), grid, dim3(256), 0, s, P, bsrc, (const float*)src, b);
  } else {
    if (f64)
      hipLaunchKernelGGL((k_bin_atomic<double, 3>), grid, dim3(256), 0, s, P, bsrc, (const double*)src, b);
    else
      hipLaunchKernelGGL((k_bin_atomic<float, 3>), grid, dim3(256), 0, s, P, bsrc, (const float*)src, b);
  }
  return hipGetLastError();
}

hipError_t launch_update(const DevPlan& P, int epi, const double* m_in, const double* b, double* out, hipStream_t s) {
  const int64_t g = std::min<int64_t>((P.npix + 255) / 256, 4096);
  if (P.ncomp == 1)
    hipLaunchKernelGGL(k_update<1>, dim3((unsigned)g), dim3(256), 0, s, P, epi, m_in, b, out);
  else
    hipLaunchKernelGGL(k_update<3>, dim3((unsigned)g), dim3(256), 0, s, P, epi, m_in, b, out);
  return hipGetLastError();
}

hipError_t launch_interleave(const DevPlan& P, const double* m, hipStream_t s) {
  if (!P.mapi) return hipSuccess;
  const int64_t g = (P.npix + 255) / 256;
  hipLaunchKernelGGL(k_interleave, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, s, P, m);
  return hipGetLastError();
}

template <typename T, int NC>
static void launch_project_t(const DevPlan& P, const double* m, T* pm_out, size_t lds, hipStream_t s) {
#define MM_PROJ(PKV)                                                                                              \
  do {                                                                                                            \
    if (P.composite)                                                                                              \
      hipLaunchKernelGGL((k_project<T, NC, PKV, true>), dim3(grid_for(P.ntiles, kGridCap)), dim3(kBinBlock), lds, \
                         s, P, m, pm_out);                                                                        \
    else                                                                                                          \
      hipLaunchKernelGGL((k_project<T, NC, PKV, false>), dim3(grid_for(P.ntiles, kGridCap)), dim3(kBinBlock),     \
                         lds, s, P, m, pm_out);                                                                   \
  } while (0)
  if constexpr (NC == 1) {
    MM_PROJ(0);
  } else {
    switch (P.psi_kind) {
      case 1: MM_PROJ(1); break;
      case 2: MM_PROJ(2); break;
      default: MM_PROJ(3); break;
    }
  }
#undef MM_PROJ
}

hipError_t launch_project(const DevPlan& P, const double* m, void* pm_out, hipStream_t s) {
  const bool f64 = P.precision == 0;
  if (P.ncomp == 1) {
    const size_t lds = f64 ? bin_lds_bytes<1, double>(false, P.max_tile_pix, false)
                           : bin_lds_bytes<1, float>(false, P.max_tile_pix, false);
    if (f64)
      launch_project_t<double, 1>(P, m, (double*)pm_out, lds, s);
    else
      launch_project_t<float, 1>(P, m, (float*)pm_out, lds, s);
  } else {
    const size_t lds = f64 ? bin_lds_bytes<3, double>(false, P.max_tile_pix, false)
                           : bin_lds_bytes<3, float>(false, P.max_tile_pix, false);
    if (f64)
      launch_project_t<double, 3>(P, m, (double*)pm_out, lds, s);
    else
      launch_project_t<float, 3>(P, m, (float*)pm_out, lds, s);
  }
  return hipGetLastError();
}

size_t binning_lds_bytes(int ncomp, int precision, int tile_pix) {
  const bool f64 = precision == 0;
  const size_t plan = ncomp == 1 ? (f64 ? bin_lds_bytes<2, double>(true, tile_pix, true)
                                        : bin_lds_bytes<2, float>(true, tile_pix, true))
                                 : (f64 ? bin_lds_bytes<7, double>(true, tile_pix, true)
                                        : bin_lds_bytes<7, float>(true, tile_pix, true));
  const size_t it = ncomp == 1 ? (f64 ? bin_lds_bytes<1, double>(false, tile_pix, true)
                                      : bin_lds_bytes<1, float>(false, tile_pix, true))
                               : (f64 ? bin_lds_bytes<3, double>(false, tile_pix, true)
                                      : bin_lds_bytes<3, float>(false, tile_pix, true));
  return plan > it ? plan : it;
}

hipError_t launch_bin(const DevPlan& P, int bsrc, const void* src, int epi, const double* m_in, double* out,
                      double* w_out, int32_t* hits_out, hipStream_t s, void* pm_out) {
  uint8_t* sol_out = reinterpret_cast<uint8_t*>(out);  // plan mode: the solvable mask
  const bool f64 = P.precision == 0;
  if (epi == EPI_PLAN) {
    if (P.ncomp == 1)
      return f64 ? launch_bin_t<double, 2>(P, bsrc, src, epi, m_in, nullptr, w_out, hits_out, sol_out, s, nullptr)
                 : launch_bin_t<float, 2>(P, bsrc, src, epi, m_in, nullptr, w_out, hits_out, sol_out, s, nullptr);
    return f64 ? launch_bin_t<double, 7>(P, bsrc, src, epi, m_in, nullptr, w_out, hits_out, sol_out, s, nullptr)
               : launch_bin_t<float, 7>(P, bsrc, src, epi, m_in, nullptr, w_out, hits_out, sol_out, s, nullptr);
  }
  if (P.ncomp == 1)
    return f64 ? launch_bin_t<double, 1>(P, bsrc, src, epi, m_in, out, w_out, hits_out, nullptr, s, pm_out)
               : launch_bin_t<float, 1>(P, bsrc, src, epi, m_in, out, w_out, hits_out, nullptr, s, pm_out);
  return f64 ? launch_bin_t<double, 3>(P, bsrc, src, epi, m_in, out, w_out, hits_out, nullptr, s, pm_out)
             : launch_bin_t<float, 3>(P, bsrc, src, epi, m_in, out, w_out, hits_out, nullptr, s, pm_out);
}

hipError_t launch_chi2_reduce(const int32_t* chunk_item_begin, const double* part, int nchunk, double* per_chunk,
                              double* total, hipStream_t s) {
  hipLaunchKernelGGL(k_chi2_reduce, dim3(1), dim3(kBlock), 0, s, chunk_item_begin, part, nchunk, per_chunk, total);
  return hipGetLastError();
}

static inline int vgrid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(vgrid(n)), dim3(256), 0, s, x, n, v);
  return hipGetLastError();
}
hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(vgrid(n)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}
hipError_t launch_copy_bytes(void* dst, const void* src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_bytes, dim3(vgrid(n)), dim3(256), 0, s, (uint8_t*)dst, (const uint8_t*)src, n);
  return hipGetLastError();
}
hipError_t launch_sub(double* out, const double* a, const double* b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_sub, dim3(vgrid(n)), dim3(256), 0, s, out, a, b, n);
  return hipGetLastError();
}
int dot_blocks(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  return (int)g;
}
hipError_t launch_dot_partials(const double* a, const double* b, int64_t n, double* part, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partials, dim3(nblk), dim3(kBlock), 0, s, a, b, n, part);
  return hipGetLastError();
}
hipError_t launch_reduce(const double* part, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, part, n, out);
  return hipGetLastError();
}
hipError_t launch_winv_apply(const DevPlan& P, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_winv_apply, dim3(vgrid(P.npix)), dim3(256), 0, s, P, x, y);
  return hipGetLastError();
}
hipError_t launch_cg_update_xr(const DevPlan& P, double* x, double* r, double* z, const double* p, const double* q,
                               const double* rz, const double* pq, double* part, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update_xr, dim3(nblk), dim3(kBlock), 0, s, P, x, r, z, p, q, rz, pq, part);
  return hipGetLastError();
}
hipError_t launch_cg_update_p(double* p, const double* z, const double* rz_new, const double* rz_old, int64_t n,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update_p, dim3(vgrid(n)), dim3(256), 0, s, p, z, rz_new, rz_old, n);
  return hipGetLastError();
}
hipError_t launch_cg_chi2(const double* chi2_0, const double* xb, const double* xr, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_chi2, dim3(1), dim3(64), 0, s, chi2_0, xb, xr, out);
  return hipGetLastError();
}

}  // namespace mm
