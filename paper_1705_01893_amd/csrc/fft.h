// LDS-resident mixed-radix Stockham transforms for gfx950.
//
// A workgroup holds `nb` independent length-L complex sequences in LDS; element i of
// sequence b lives at lds[i * nb + b] (interleaved columns, nb a power of two) or at
// lds[b * L + i] (consecutive rows, nb <= 4).  One radix-R stage reads every element
// into registers (R per butterfly, a fixed number of butterflies per thread),
// synchronises, applies twiddles and the R-point DFT in registers, and
// writes the results to their self-sorting (Stockham) positions; after the last
// stage the sequences are in natural frequency order in place.  Radices 2, 3, 4,
// 5 and 8 cover every 5-smooth length; the composite radices 9, 16, 20 and 25
// (two-level DFTs in registers) cut the number of stages where the register
// budget allows them (radix_ok).
#pragma once

#include "common.h"

namespace mm {

template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename C>
__device__ __forceinline__ C cadd(C a, C b) {
  C r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <typename C>
__device__ __forceinline__ C csub(C a, C b) {
  C r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C>
__device__ __forceinline__ C rot(C a) {
  C r;
  if (INV) {
    r.x = -a.y;
    r.y = a.x;
  } else {
    r.x = a.y;
    r.y = -a.x;
  }
  return r;
}
template <typename C, typename T>
__device__ __forceinline__ C cscale(C a, T s) {
  C r;
  r.x = a.x * s;
  r.y = a.y * s;
  return r;
}

// In-register R-point DFT, forward (exp(-2 pi i jk/R)) or inverse (exp(+...)), unnormalised.
template <typename T, int R, bool INV>
struct Dft;

template <typename T, bool INV>
struct Dft<T, 2, INV> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    cx<T> t = a[1];
    a[1] = csub(a[0], t);
    a[0] = cadd(a[0], t);
  }
};

template <typename T, bool INV>
struct Dft<T, 4, INV> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    cx<T> t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    cx<T> t2 = cadd(a[1], a[3]), t3 = rot<INV>(csub(a[1], a[3]));
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
  }
};

template <typename T, bool INV>
struct Dft<T, 8, INV> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    cx<T> e[4] = {a[0], a[2], a[4], a[6]};
    cx<T> o[4] = {a[1], a[3], a[5], a[7]};
    Dft<T, 4, INV>::run(e);
    Dft<T, 4, INV>::run(o);
    const T h = T(0.70710678118654752440084436210484903928);
    // o[k] *= w8^k, w8 = exp(-+ i pi/4)
    cx<T> o1, o3;
    if (INV) {
      o1.x = h * (o[1].x - o[1].y);
      o1.y = h * (o[1].x + o[1].y);
      o3.x = -h * (o[3].x + o[3].y);
      o3.y = h * (o[3].x - o[3].y);
    } else {
      o1.x = h * (o[1].x + o[1].y);
      o1.y = h * (o[1].y - o[1].x);
      o3.x = h * (o[3].y - o[3].x);
      o3.y = -h * (o[3].x + o[3].y);
    }
    cx<T> o2 = rot<INV>(o[2]);
    a[0] = cadd(e[0], o[0]);
    a[4] = csub(e[0], o[0]);
    a[1] = cadd(e[1], o1);
    a[5] = csub(e[1], o1);
    a[2] = cadd(e[2], o2);
    a[6] = csub(e[2], o2);
    a[3] = cadd(e[3], o3);
    a[7] = csub(e[3], o3);
  }
};

template <typename T, bool INV>
struct Dft<T, 3, INV> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    const T s3 = T(0.86602540378443864676372317075293618347);
    cx<T> t = cadd(a[1], a[2]);
    cx<T> u = csub(a[0], cscale(t, T(0.5)));
    cx<T> v = rot<INV>(cscale(csub(a[1], a[2]), s3));
    a[0] = cadd(a[0], t);
    a[1] = cadd(u, v);
    a[2] = csub(u, v);
  }
};

template <typename T, bool INV>
struct Dft<T, 5, INV> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    const T c1 = T(0.30901699437494742410229341718281905886);   // cos(2 pi/5)
    const T c2 = T(-0.80901699437494742410229341718281905886);  // cos(4 pi/5)
    const T s1 = T(0.95105651629515357211643933337938214340);   // sin(2 pi/5)
    const T s2 = T(0.58778525229247312916870595463907276860);   // sin(4 pi/5)
    cx<T> b1 = cadd(a[1], a[4]), b2 = cadd(a[2], a[3]);
    cx<T> d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
    cx<T> x0 = a[0];
    cx<T> p1 = cadd(x0, cadd(cscale(b1, c1), cscale(b2, c2)));
    cx<T> p2 = cadd(x0, cadd(cscale(b1, c2), cscale(b2, c1)));
    cx<T> q1 = rot<INV>(cadd(cscale(d1, s1), cscale(d2, s2)));
    cx<T> q2 = rot<INV>(csub(cscale(d1, s2), cscale(d2, s1)));
    a[0] = cadd(x0, cadd(b1, b2));
    a[1] = cadd(p1, q1);
    a[4] = csub(p1, q1);
    a[2] = cadd(p2, q2);
    a[3] = csub(p2, q2);
  }
};

// cos and sin of 2 pi e / R for the composite radices, correctly rounded (e folded into [0, R/2]
// by symmetry)
template <int R>
__device__ __forceinline__ void root_cs(int e, double& c, double& s) {
  e %= R;
  const bool neg = 2 * e > R;
  if (neg) e = R - e;
  c = 1.0;
  s = 0.0;
  switch (R) {
    case 6:
      switch (e) {
        case 1: c = 0.5; s = 0.8660254037844386; break;
        case 2: c = -0.5; s = 0.8660254037844386; break;
        case 3: c = -1.0; s = 0.0; break;
        default: break;
      }
      break;
    case 9:
      switch (e) {
        case 1: c = 0.766044443118978; s = 0.6427876096865394; break;
        case 2: c = 0.17364817766693036; s = 0.984807753012208; break;
        case 3: c = -0.5; s = 0.8660254037844386; break;
        case 4: c = -0.9396926207859084; s = 0.3420201433256687; break;
        default: break;
      }
      break;
    case 10:
      switch (e) {
        case 1: c = 0.8090169943749475; s = 0.5877852522924731; break;
        case 2: c = 0.30901699437494745; s = 0.9510565162951535; break;
        case 3: c = -0.30901699437494745; s = 0.9510565162951535; break;
        case 4: c = -0.8090169943749475; s = 0.5877852522924731; break;
        case 5: c = -1.0; s = 0.0; break;
        default: break;
      }
      break;
    case 12:
      switch (e) {
        case 1: c = 0.8660254037844386; s = 0.5; break;
        case 2: c = 0.5; s = 0.8660254037844386; break;
        case 3: c = 0.0; s = 1.0; break;
        case 4: c = -0.5; s = 0.8660254037844386; break;
        case 5: c = -0.8660254037844386; s = 0.5; break;
        case 6: c = -1.0; s = 0.0; break;
        default: break;
      }
      break;
    case 15:
      switch (e) {
        case 1: c = 0.9135454576426009; s = 0.4067366430758002; break;
        case 2: c = 0.6691306063588582; s = 0.7431448254773942; break;
        case 3: c = 0.30901699437494745; s = 0.9510565162951535; break;
        case 4: c = -0.10452846326765347; s = 0.9945218953682733; break;
        case 5: c = -0.5; s = 0.8660254037844386; break;
        case 6: c = -0.8090169943749475; s = 0.5877852522924731; break;
        case 7: c = -0.9781476007338057; s = 0.20791169081775934; break;
        default: break;
      }
      break;
    case 16:
      switch (e) {
        case 1: c = 0.9238795325112867; s = 0.3826834323650898; break;
        case 2: c = 0.7071067811865476; s = 0.7071067811865476; break;
        case 3: c = 0.3826834323650898; s = 0.9238795325112867; break;
        case 4: c = 0.0; s = 1.0; break;
        case 5: c = -0.3826834323650898; s = 0.9238795325112867; break;
        case 6: c = -0.7071067811865476; s = 0.7071067811865476; break;
        case 7: c = -0.9238795325112867; s = 0.3826834323650898; break;
        case 8: c = -1.0; s = 0.0; break;
        default: break;
      }
      break;
    case 20:
      switch (e) {
        case 1: c = 0.9510565162951535; s = 0.30901699437494745; break;
        case 2: c = 0.8090169943749475; s = 0.5877852522924731; break;
        case 3: c = 0.5877852522924731; s = 0.8090169943749475; break;
        case 4: c = 0.30901699437494745; s = 0.9510565162951535; break;
        case 5: c = 0.0; s = 1.0; break;
        case 6: c = -0.30901699437494745; s = 0.9510565162951535; break;
        case 7: c = -0.5877852522924731; s = 0.8090169943749475; break;
        case 8: c = -0.8090169943749475; s = 0.5877852522924731; break;
        case 9: c = -0.9510565162951535; s = 0.30901699437494745; break;
        case 10: c = -1.0; s = 0.0; break;
        default: break;
      }
      break;
    case 25:
      switch (e) {
        case 1: c = 0.9685831611286311; s = 0.2486898871648548; break;
        case 2: c = 0.8763066800438636; s = 0.48175367410171527; break;
        case 3: c = 0.7289686274214116; s = 0.6845471059286887; break;
        case 4: c = 0.5358267949789967; s = 0.8443279255020151; break;
        case 5: c = 0.30901699437494745; s = 0.9510565162951535; break;
        case 6: c = 0.06279051952931337; s = 0.9980267284282716; break;
        case 7: c = -0.18738131458572463; s = 0.9822872507286887; break;
        case 8: c = -0.42577929156507266; s = 0.9048270524660196; break;
        case 9: c = -0.6374239897486897; s = 0.7705132427757893; break;
        case 10: c = -0.8090169943749475; s = 0.5877852522924731; break;
        case 11: c = -0.9297764858882515; s = 0.368124552684678; break;
        case 12: c = -0.9921147013144779; s = 0.12533323356430426; break;
        default: break;
      }
      break;
    default: break;
  }
  if (neg) s = -s;
}

// R = R1 R2 point DFT from R1- and R2-point ones: with n = R2 n1 + n2 and k = k1 + R1 k2,
// X_k = sum_n2 W_R^(n2 k1) W_R2^(n2 k2) sum_n1 a_n W_R1^(n1 k1) (W_R = exp(-+ 2 pi i / R)):
// R2 inner transforms over n1, the R1 R2 twiddles, R1 outer transforms over n2.
template <typename T, int R1, int R2, bool INV>
struct Dft2 {
  __device__ __forceinline__ static void run(cx<T>* a) {
    constexpr int R = R1 * R2;
    cx<T> b[R2][R1];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) b[n2][n1] = a[R2 * n1 + n2];
      Dft<T, R1, INV>::run(b[n2]);
    }
#pragma unroll
    for (int n2 = 1; n2 < R2; ++n2)
#pragma unroll
      for (int k1 = 1; k1 < R1; ++k1) {
        double c, s;
        root_cs<R>(n2 * k1, c, s);
        cx<T> w;
        w.x = T(c);
        w.y = INV ? T(s) : T(-s);
        b[n2][k1] = cmul(b[n2][k1], w);
      }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      cx<T> t[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) t[n2] = b[n2][k1];
      Dft<T, R2, INV>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) a[k1 + R1 * k2] = t[k2];
    }
  }
};

// composite radices R = R1 R2 (Split<R>: the factors; R2 is also the inner step of the twiddles)
template <int R>
struct Split {
  static constexpr int r1 = 0, r2 = 0;
};
#define MM_SPLIT(R, A, B)                  \
  template <>                              \
  struct Split<R> {                        \
    static constexpr int r1 = A, r2 = B;   \
  };                                       \
  template <typename T, bool INV>          \
  struct Dft<T, R, INV> {                  \
    __device__ __forceinline__ static void run(cx<T>* a) { Dft2<T, A, B, INV>::run(a); } \
  };
MM_SPLIT(6, 2, 3)
MM_SPLIT(9, 3, 3)
MM_SPLIT(10, 2, 5)
MM_SPLIT(12, 4, 3)
MM_SPLIT(15, 3, 5)
MM_SPLIT(16, 4, 4)
MM_SPLIT(20, 4, 5)
MM_SPLIT(25, 5, 5)
#undef MM_SPLIT

// Exact quotient n / d for n, d < 2^22 from a single-precision reciprocal estimate
// (the estimate is within one of the quotient, corrected with one multiply-subtract).
__device__ __forceinline__ uint32_t qdiv(uint32_t n, uint32_t d, float inv) {
  uint32_t q = (uint32_t)((float)n * inv);
  const int32_t r = (int32_t)(n - q * d);
  if (r < 0)
    --q;
  else if (r >= (int32_t)d)
    ++q;
  return q;
}

// w^m for m = 0..R-1 from w = v[1] by balanced products (error grows like log2 m ulps); for a
// composite radix R = R1 R2, w^m = w^(m mod R2) (w^R2)^(m div R2), which keeps R1 + R2 powers
// live instead of R - 1
template <typename T, int R>
__device__ __forceinline__ void twiddle_powers(cx<T>* v, cx<T> w1) {
  constexpr int B = Split<R>::r2, A = Split<R>::r1;
  if constexpr (B > 0) {
    cx<T> lo[B], hi[A];
    lo[0].x = T(1);
    lo[0].y = T(0);
    lo[1] = w1;
#pragma unroll
    for (int m = 2; m < B; ++m) lo[m] = (m % 2 == 0) ? cmul(lo[m / 2], lo[m / 2]) : cmul(lo[m - 1], w1);
    hi[0] = lo[0];
    hi[1] = cmul(lo[B - 1], w1);
#pragma unroll
    for (int m = 2; m < A; ++m) hi[m] = (m % 2 == 0) ? cmul(hi[m / 2], hi[m / 2]) : cmul(hi[m - 1], hi[1]);
#pragma unroll
    for (int m = 1; m < R; ++m) {
      const int j = m % B, q = m / B;
      const cx<T> w = (q == 0) ? lo[j] : (j == 0 ? hi[q] : cmul(hi[q], lo[j]));
      v[m] = cmul(v[m], w);
    }
    return;
  }
  cx<T> w[R];
  w[1] = w1;
#pragma unroll
  for (int m = 2; m < R; ++m) w[m] = (m % 2 == 0) ? cmul(w[m / 2], w[m / 2]) : cmul(w[m - 1], w1);
#pragma unroll
  for (int m = 1; m < R; ++m) v[m] = cmul(v[m], w[m]);
}

// One Stockham stage run by a workgroup of NT threads.  p = product of the radices already
// applied.  Butterfly f of the stage belongs to sequence b and position k: with BFAST,
// b = f mod nb (nb a power of two, lg_nb = log2 nb), otherwise b = f / (L/R) with nb <= 4.
// Kept out of line: inlining all five radix variants into the stage loop makes the register
// allocator budget for their union and halves the occupancy of every pass.
// LDS and global pointers with their address spaces spelled out (32-bit LDS address arithmetic
// and ds_* instructions; global, not flat, loads of the twiddle tables), over a plain two-lane
// vector type so that loads and stores stay single vector instructions.
template <typename T>
using vec2 = T __attribute__((ext_vector_type(2)));
template <typename T>
using lds_v2 = __attribute__((address_space(3))) vec2<T>*;
template <typename T>
using glob_v2 = const __attribute__((address_space(1))) vec2<T>*;

template <typename T>
__device__ __forceinline__ cx<T> to_cx(vec2<T> a) {
  cx<T> r;
  r.x = a.x;
  r.y = a.y;
  return r;
}
template <typename T>
__device__ __forceinline__ vec2<T> to_v2(cx<T> a) {
  vec2<T> r;
  r.x = a.x;
  r.y = a.y;
  return r;
}

template <typename T, int R, bool INV, bool BFAST, int NT>
__device__ __forceinline__ void stage_body(cx<T>* lds_generic, int L, int nb, int lg_nb, int p,
                                           const cx<T>* __restrict__ tw_generic) {
  const lds_v2<T> lds = (lds_v2<T>)lds_generic;
  const glob_v2<T> tw = (glob_v2<T>)tw_generic;
  constexpr int K = (Ept<T>::v + R - 1) / R;  // butterflies per thread
  const int nbf = L / R;
  const int total = nbf * nb;
  const int step = L / (p * R);
  // element i of sequence b sits at i * sI + b * sB: interleaved columns (BFAST: sI = nb, sB = 1)
  // or consecutive rows (sI = 1, sB = L)
  const int sI = BFAST ? (1 << lg_nb) : 1;
  const int sB = BFAST ? 1 : L;
  const int rstride = nbf * sI;  // LDS distance between the R inputs of a butterfly
  const int wstride = p * sI;    // and between its R outputs
  const float inv_p = 1.0f / (float)p;
  cx<T> v[K][R];
  int bk[K][2];
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int f = threadIdx.x + u * NT;
    int b = 0, k = 0;
    if (BFAST) {
      b = f & (nb - 1);
      k = f >> lg_nb;
    } else {
      // the row transforms hold at most four sequences: b = f / nbf by comparisons
      b = (f >= nbf) + (f >= 2 * nbf) + (f >= 3 * nbf);
      k = f - b * nbf;
    }
    bk[u][0] = b;
    bk[u][1] = k;
    if (f < total) {
      int a = k * sI + b * sB;
#pragma unroll
      for (int m = 0; m < R; ++m, a += rstride) v[u][m] = to_cx<T>(lds[a]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int f = threadIdx.x + u * NT;
    if (f < total) {
      const int b = bk[u][0], k = bk[u][1];
      const int kq = (int)qdiv((uint32_t)k, (uint32_t)p, inv_p);
      const int j = k - kq * p;
      if (j != 0) {
        cx<T> w = to_cx<T>(tw[j * step]);
        if (INV) w.y = -w.y;
        twiddle_powers<T, R>(v[u], w);
      }
      Dft<T, R, INV>::run(v[u]);
      int a = (kq * p * R + j) * sI + b * sB;
#pragma unroll
      for (int m = 0; m < R; ++m, a += wstride) lds[a] = to_v2<T>(v[u][m]);
    }
  }
  __syncthreads();
}

template <typename T, int R, bool INV, bool BFAST, int NT>
__device__ __attribute__((noinline)) void stockham_stage(cx<T>* lds, int L, int nb, int lg_nb, int p,
                                               const cx<T>* __restrict__ tw) {
  stage_body<T, R, INV, BFAST, NT>(lds, L, nb, lg_nb, p, tw);
}

// Full length-L transform of nb sequences (caller synchronises before the first stage).
// tw: omega_L^q = exp(-2 pi i q / L), q < L.  Each stage is a call: a callee waits for all
// of the caller's outstanding memory operations on entry.
template <typename T, bool INV, bool BFAST, int NT>
__device__ void lds_fft(cx<T>* lds, int L, int nb, int lg_nb, const int8_t* rad, int ns,
                        const cx<T>* __restrict__ tw) {
  int p = 1;
  for (int s = 0; s < ns; ++s) {
    const int R = rad[s];
    switch (R) {
      case 8: stockham_stage<T, 8, INV, BFAST, NT>(lds, L, nb, lg_nb, p, tw); break;
      case 4: stockham_stage<T, 4, INV, BFAST, NT>(lds, L, nb, lg_nb, p, tw); break;
      case 2: stockham_stage<T, 2, INV, BFAST, NT>(lds, L, nb, lg_nb, p, tw); break;
      case 3: stockham_stage<T, 3, INV, BFAST, NT>(lds, L, nb, lg_nb, p, tw); break;
      case 5: stockham_stage<T, 5, INV, BFAST, NT>(lds, L, nb, lg_nb, p, tw); break;
      // composite radices, where the precision's schedules use them
      case 6:
        if constexpr (radix_ok(6, sizeof(T) == 8)) stockham_stage<T, 6, INV, BFAST, NT>(lds, L, nb, lg_nb, p, tw);
        break;
      case 9:
        if constexpr (radix_ok(9, sizeof(T) == 8)) stockham_stage<T, 9, INV, BFAST, NT>(lds, L, nb, lg_nb, p, tw);
        break;
      case 10:
        if constexpr (radix_ok(10, sizeof(T) == 8)) stockham_stage<T, 10, INV, BFAST, NT>(lds, L, nb, lg_nb, p, tw);
        break;
      case 12:
        if constexpr (radix_ok(12, sizeof(T) == 8)) stockham_stage<T, 12, INV, BFAST, NT>(lds, L, nb, lg_nb, p, tw);
        break;
      case 15:
        if constexpr (radix_ok(15, sizeof(T) == 8)) stockham_stage<T, 15, INV, BFAST, NT>(lds, L, nb, lg_nb, p, tw);
        break;
      case 16:
        if constexpr (radix_ok(16, sizeof(T) == 8)) stockham_stage<T, 16, INV, BFAST, NT>(lds, L, nb, lg_nb, p, tw);
        break;
      case 20:
        if constexpr (radix_ok(20, sizeof(T) == 8)) stockham_stage<T, 20, INV, BFAST, NT>(lds, L, nb, lg_nb, p, tw);
        break;
      case 25:
        if constexpr (radix_ok(25, sizeof(T) == 8)) stockham_stage<T, 25, INV, BFAST, NT>(lds, L, nb, lg_nb, p, tw);
        break;
      default: break;
    }
    p *= R;
  }
}

// One Stockham stage of NB sequences of length L, every size known at compile time (p = P, the
// product of the radices applied before): the sequence and position of each butterfly, the
// quotient k / P and the LDS strides fold into shifts and immediate offsets.  Element i of
// sequence b sits at b L + i (consecutive rows; butterfly f in sequence f / (L / R)) or, with
// BFAST, at i NB + b (interleaved columns; butterfly f in sequence f mod NB).
template <typename T, int R, bool INV, int L, int NB, int P, int NT, bool BFAST = false>
__device__ __attribute__((noinline)) void stage_ct(cx<T>* lds_generic, const cx<T>* __restrict__ tw_generic) {
  const lds_v2<T> lds = (lds_v2<T>)lds_generic;
  const glob_v2<T> tw = (glob_v2<T>)tw_generic;
  constexpr int NBF = L / R, TOTAL = NBF * NB, STEP = L / (P * R), K = TOTAL / NT;
  constexpr int SI = BFAST ? NB : 1, SB = BFAST ? 1 : L;
  static_assert(TOTAL % NT == 0 && (NBF & (NBF - 1)) == 0 && (P & (P - 1)) == 0 && (NB & (NB - 1)) == 0,
                "power-of-two stage");
  cx<T> v[K][R];
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int f = (int)threadIdx.x + u * NT;
    const int b = BFAST ? f % NB : f / NBF, k = BFAST ? f / NB : f % NBF;
#pragma unroll
    for (int m = 0; m < R; ++m) v[u][m] = to_cx<T>(lds[b * SB + (k + m * NBF) * SI]);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int f = (int)threadIdx.x + u * NT;
    const int b = BFAST ? f % NB : f / NBF, k = BFAST ? f / NB : f % NBF;
    const int kq = k / P, j = k % P;
    if (P > 1 && j != 0) {
      cx<T> w = to_cx<T>(tw[j * STEP]);
      if (INV) w.y = -w.y;
      twiddle_powers<T, R>(v[u], w);
    }
    Dft<T, R, INV>::run(v[u]);
#pragma unroll
    for (int m = 0; m < R; ++m) lds[b * SB + (kq * P * R + j + m * P) * SI] = to_v2<T>(v[u][m]);
  }
  __syncthreads();
}

// Whether a row item runs the precision's compiled-in schedule: two rows of 2048 points under
// radices 8, 16, 16 in FP32, of 1024 points under 4, 4, 8, 8 in FP64.
template <typename T>
__device__ __forceinline__ bool row_ct_ok(int M1, int nrow, int nr, const int8_t* rad) {
  if (nrow != 2) return false;
  if (sizeof(T) == 4) return M1 == 2048 && nr == 3 && rad[0] == 8 && rad[1] == 16 && rad[2] == 16;
  return M1 == 1024 && nr == 4 && rad[0] == 4 && rad[1] == 4 && rad[2] == 8 && rad[3] == 8;
}

// The transform of lds_fft for power-of-two lengths (radices 8, 4 and 2 only), with the stages
// inlined: no call boundaries, so loads the caller has in flight stay in flight.
template <typename T, bool INV, bool BFAST, int NT>
__device__ __forceinline__ void lds_fft_pow2(cx<T>* lds, int L, int nb, int lg_nb, const int8_t* rad, int ns,
                                             const cx<T>* __restrict__ tw) {
  int p = 1;
#pragma unroll 1
  for (int s = 0; s < ns; ++s) {
    const int R = rad[s];
    if (R == 8)
      stage_body<T, 8, INV, BFAST, NT>(lds, L, nb, lg_nb, p, tw);
    else if (R == 4)
      stage_body<T, 4, INV, BFAST, NT>(lds, L, nb, lg_nb, p, tw);
    else
      stage_body<T, 2, INV, BFAST, NT>(lds, L, nb, lg_nb, p, tw);
    p *= R;
  }
}

// ---------------------------------------------------------------------------------------------
// Wave-local transforms: one wave transforms nw sequences of length L on its own, sequence c at
// cols + c * Lc with element i at pad8(i) (one spare slot per eight keeps the stride-R outputs
// of a stage in distinct banks).  Butterfly f of a stage belongs to sequence c = f / (L/R) and
// position k = f mod (L/R), so consecutive lanes read consecutive elements.  A wave's LDS
// operations are performed in order, so the stages need only a wave-scope fence (which also
// keeps the compiler from moving LDS accesses across it), no workgroup barrier.

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void wave_stage_body(cx<T>* cols_generic, int L, int Lc, int nw, int p,
                                                const cx<T>* __restrict__ tw_generic) {
  const lds_v2<T> cols = (lds_v2<T>)cols_generic;
  const glob_v2<T> tw = (glob_v2<T>)tw_generic;
  constexpr int K = (Ept<T>::v + R - 1) / R;  // butterflies per lane
  const int lane = (int)(threadIdx.x & 63);
  const int nbf = L / R;
  const int total = nbf * nw;
  const int step = L / (p * R);
  const float inv_p = 1.0f / (float)p, inv_n = 1.0f / (float)nbf;
  cx<T> v[K][R];
  int ck[K][2];
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int f = lane + u * 64;
    const int c = (int)qdiv((uint32_t)f, (uint32_t)nbf, inv_n);
    const int k = f - c * nbf;
    ck[u][0] = c * Lc;
    ck[u][1] = k;
    if (f < total) {
#pragma unroll
      for (int m = 0; m < R; ++m) v[u][m] = to_cx<T>(cols[ck[u][0] + pad8(k + m * nbf)]);
    }
  }
  wave_sync();
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int f = lane + u * 64;
    if (f < total) {
      const int k = ck[u][1];
      const int kq = (int)qdiv((uint32_t)k, (uint32_t)p, inv_p);
      const int j = k - kq * p;
      if (j != 0) {
        cx<T> w = to_cx<T>(tw[j * step]);
        if (INV) w.y = -w.y;
        twiddle_powers<T, R>(v[u], w);
      }
      Dft<T, R, INV>::run(v[u]);
      const int o = kq * p * R + j;
#pragma unroll
      for (int m = 0; m < R; ++m) cols[ck[u][0] + pad8(o + m * p)] = to_v2<T>(v[u][m]);
    }
  }
  wave_sync();
}

template <typename T, int R, bool INV>
__device__ __attribute__((noinline)) void wave_stockham_stage(cx<T>* cols, int L, int Lc, int nw, int p,
                                                              const cx<T>* __restrict__ tw) {
  wave_stage_body<T, R, INV>(cols, L, Lc, nw, p, tw);
}

// Full transform of the calling wave's nw sequences (L * nw <= 64 * Ept<T>); the caller
// synchronises the workgroup before (the sequences are loaded) and after (other waves read
// them).
template <typename T, bool INV>
__device__ __forceinline__ void wave_fft(cx<T>* cols, int L, int Lc, int nw, const int8_t* rad, int ns,
                                         const cx<T>* __restrict__ tw) {
  int p = 1;
#pragma unroll 1
  for (int s = 0; s < ns; ++s) {
    const int R = rad[s];
    switch (R) {
      case 8: wave_stockham_stage<T, 8, INV>(cols, L, Lc, nw, p, tw); break;
      case 4: wave_stockham_stage<T, 4, INV>(cols, L, Lc, nw, p, tw); break;
      case 2: wave_stockham_stage<T, 2, INV>(cols, L, Lc, nw, p, tw); break;
      case 3: wave_stockham_stage<T, 3, INV>(cols, L, Lc, nw, p, tw); break;
      case 5: wave_stockham_stage<T, 5, INV>(cols, L, Lc, nw, p, tw); break;
      case 6:
        if constexpr (radix_ok(6, sizeof(T) == 8)) wave_stockham_stage<T, 6, INV>(cols, L, Lc, nw, p, tw);
        break;
      case 9:
        if constexpr (radix_ok(9, sizeof(T) == 8)) wave_stockham_stage<T, 9, INV>(cols, L, Lc, nw, p, tw);
        break;
      case 10:
        if constexpr (radix_ok(10, sizeof(T) == 8)) wave_stockham_stage<T, 10, INV>(cols, L, Lc, nw, p, tw);
        break;
      case 12:
        if constexpr (radix_ok(12, sizeof(T) == 8)) wave_stockham_stage<T, 12, INV>(cols, L, Lc, nw, p, tw);
        break;
      case 15:
        if constexpr (radix_ok(15, sizeof(T) == 8)) wave_stockham_stage<T, 15, INV>(cols, L, Lc, nw, p, tw);
        break;
      case 16:
        if constexpr (radix_ok(16, sizeof(T) == 8)) wave_stockham_stage<T, 16, INV>(cols, L, Lc, nw, p, tw);
        break;
      case 20:
        if constexpr (radix_ok(20, sizeof(T) == 8)) wave_stockham_stage<T, 20, INV>(cols, L, Lc, nw, p, tw);
        break;
      case 25:
        if constexpr (radix_ok(25, sizeof(T) == 8)) wave_stockham_stage<T, 25, INV>(cols, L, Lc, nw, p, tw);
        break;
      default: break;
    }
    p *= R;
  }
}

// ---------------------------------------------------------------------------------------------
// Register-resident transform of 1024 FP32 points held by one wave, lane l holding elements
// l + 64 i (i < 16) in v[i]: a 16-point DFT over each lane's values, the twiddles
// omega_1024^(l k1), then a 64-point decimation-in-frequency transform across the lanes, one
// radix-2 level per lane bit, the partners exchanged by lane shuffles (DPP for lane xor 1 and 2,
// ds_swizzle for xor 4, 8 and 16, v_permlane32_swap for xor 32) instead of LDS round trips.
// On return lane l, register k1 holds X[k1 + 16 rev6(l)] (rev6: the reversal of l's six bits).
// tw: omega_1024^q, q < 1024.

// x of lane (lane xor h); h a compile-time constant after unrolling
__device__ __forceinline__ float lane_xor(float x, int h) {
  const int xi = __float_as_int(x);
  int r;
  if (h == 1) {
    r = __builtin_amdgcn_mov_dpp(xi, 0xB1, 0xF, 0xF, false);  // quad_perm [1, 0, 3, 2]
  } else if (h == 2) {
    r = __builtin_amdgcn_mov_dpp(xi, 0x4E, 0xF, 0xF, false);  // quad_perm [2, 3, 0, 1]
  } else if (h == 4) {
    r = __builtin_amdgcn_ds_swizzle(xi, 0x101F);  // bit mode: and mask 0x1f, xor mask h
  } else if (h == 8) {
    r = __builtin_amdgcn_ds_swizzle(xi, 0x201F);
  } else if (h == 16) {
    r = __builtin_amdgcn_ds_swizzle(xi, 0x401F);
  } else {
    // v_permlane32_swap: the upper half of the first operand trades places with the lower half
    // of the second, so lane l >= 32 finds lane l - 32 in the first, lane l < 32 lane l + 32 in
    // the second
    const auto pr = __builtin_amdgcn_permlane32_swap((unsigned)xi, (unsigned)xi, false, false);
    r = (threadIdx.x & 32) ? (int)pr[0] : (int)pr[1];
  }
  return __int_as_float(r);
}

template <bool INV>
__device__ __forceinline__ void wave_fft1024_regs(cx<float>* v, const cx<float>* __restrict__ tw) {
  const int lane = (int)(threadIdx.x & 63);
  cx<float> wl = tw[lane];
  if (INV) wl.y = -wl.y;
  Dft<float, 16, INV>::run(v);
  twiddle_powers<float, 16>(v, wl);
  // the lane pair (l, l + h) of a level: a + b stays low, (a - b) omega_2h^(l mod h) goes high
  cx<float> lw[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int h = 32 >> s;
    lw[s] = tw[(lane & h) ? 16 * (lane & (h - 1)) * (32 / h) : 0];
    if (INV) lw[s].y = -lw[s].y;
  }
  // the registers' 64-point transforms are independent: one register's six levels at a time
#pragma unroll
  for (int i = 0; i < 16; ++i) {
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int h = 32 >> s;
      const float sg = (lane & h) ? -1.0f : 1.0f;
      cx<float> t;
      if (h == 32) {
        // one swap per component hands every lane both values of its pair: lane l finds
        // x[l mod 32] in the first result and x[(l mod 32) + 32] in the second
        const auto px = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i].x), __float_as_uint(v[i].x), false, false);
        const auto py = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i].y), __float_as_uint(v[i].y), false, false);
        t.x = fmaf(sg, __uint_as_float(px[1]), __uint_as_float(px[0]));
        t.y = fmaf(sg, __uint_as_float(py[1]), __uint_as_float(py[0]));
      } else {
        t.x = fmaf(sg, v[i].x, lane_xor(v[i].x, h));
        t.y = fmaf(sg, v[i].y, lane_xor(v[i].y, h));
      }
      // the low lane of a pair holds omega^0 = (1, 0): the product returns t unchanged there
      v[i] = cmul(t, lw[s]);
    }
  }
}

// The transform of one 1024-point column in LDS (element i at pad8(i), natural order in and
// out) by the calling wave.  Inlined into a kernel variant that makes no other transform calls
// (a call would make it save the callee-saved registers it uses to scratch, every item).
template <bool INV>
__device__ __forceinline__ void wave_col1024_regs(cx<float>* col, const cx<float>* __restrict__ tw) {
  const int lane = (int)(threadIdx.x & 63);
  cx<float> v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = col[pad8(lane + 64 * i)];
  wave_fft1024_regs<INV>(v, tw);
  const int br = (int)(__builtin_bitreverse32((uint32_t)lane) >> 26);
#pragma unroll
  for (int i = 0; i < 16; ++i) col[pad8(i + 16 * br)] = v[i];
}

template <typename T, bool INV, bool BFAST, int NT, bool P2>
__device__ __forceinline__ void lds_transform(cx<T>* lds, int L, int nb, int lg_nb, const int8_t* rad, int ns,
                                              const cx<T>* __restrict__ tw) {
  if (P2)
    lds_fft_pow2<T, INV, BFAST, NT>(lds, L, nb, lg_nb, rad, ns, tw);
  else
    lds_fft<T, INV, BFAST, NT>(lds, L, nb, lg_nb, rad, ns, tw);
}

}  // namespace mm
