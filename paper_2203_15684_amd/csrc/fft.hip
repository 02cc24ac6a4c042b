// Plane-wave <-> real-space transforms for gfx950.
//
// A band vector lives on a sphere of plane waves.  The 3D transform is split
// into (1) z-sticks: a direct DFT along z of every (m1, m2) column that holds
// sphere points, and (2) xy-planes: one workgroup per (band, z) keeps the whole
// N1 x N2 plane in LDS and runs in-place mixed-radix FFTs along y (only the
// columns that hold sticks) and x.  The inverse direction uses decimation in
// frequency (natural in, digit-reversed out) and the forward direction the
// exact reverse sequence (digit-reversed in, natural out), so the real-space
// side is kept in digit-reversed x/y order and no permutation pass is needed:
// the local potential, the cached occupied states, the response density and
// potential are all stored in that order.
#include <algorithm>
#include <type_traits>

#include "hp_internal.h"

namespace hp {

namespace {

constexpr int kThreads = 256;
constexpr int kStickChunk = 32;  // sticks per workgroup in the z-DFT kernels
constexpr int kMaxPerThread = 40;  // plane elements per thread kept in registers

// Complex helpers for double2 (FP64 path) and float2 (FP32 path).
template <class C>
__device__ __forceinline__ C mkc(double x, double y);
template <>
__device__ __forceinline__ double2 mkc<double2>(double x, double y) {
  return make_double2(x, y);
}
template <>
__device__ __forceinline__ float2 mkc<float2>(double x, double y) {
  return make_float2((float)x, (float)y);
}
template <class C>
__device__ __forceinline__ C czero() {
  C r;
  r.x = 0;
  r.y = 0;
  return r;
}
template <class C>
__device__ __forceinline__ C cadd(C a, C b) {
  a.x += b.x;
  a.y += b.y;
  return a;
}
template <class C>
__device__ __forceinline__ C csub(C a, C b) {
  a.x -= b.x;
  a.y -= b.y;
  return a;
}
template <class C>
__device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <class C>
__device__ __forceinline__ C cmulc(C a, C b) {  // a * conj(b)
  C r;
  r.x = a.x * b.x + a.y * b.y;
  r.y = a.y * b.x - a.x * b.y;
  return r;
}
template <class C, class S>
__device__ __forceinline__ C cscale(C a, S s) {
  using R = decltype(a.x);
  a.x *= (R)s;
  a.y *= (R)s;
  return a;
}
// multiply by sign * i
template <class C, class S>
__device__ __forceinline__ C cmul_si(C a, S sign) {
  using R = decltype(a.x);
  C r;
  r.x = -(R)sign * a.y;
  r.y = (R)sign * a.x;
  return r;
}

// y_t = sum_u x_u exp(sign 2 pi i u t / R), in registers.
template <int RDX, class C>
__device__ __forceinline__ void dft_small(C *x, double sign_d) {
  using R = decltype(x[0].x);
  const R sign = (R)sign_d;
  if constexpr (RDX == 2) {
    C a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else if constexpr (RDX == 3) {
    const R h = (R)0.86602540378443864676;  // sqrt(3)/2
    C s = cadd(x[1], x[2]);
    C d = csub(x[1], x[2]);
    C m;
    m.x = x[0].x - (R)0.5 * s.x;
    m.y = x[0].y - (R)0.5 * s.y;
    C t = cmul_si(cscale(d, h), sign);
    x[0] = cadd(x[0], s);
    x[1] = cadd(m, t);
    x[2] = csub(m, t);
  } else if constexpr (RDX == 4) {
    C a0 = cadd(x[0], x[2]), a1 = csub(x[0], x[2]);
    C b0 = cadd(x[1], x[3]), b1 = cmul_si(csub(x[1], x[3]), sign);
    x[0] = cadd(a0, b0);
    x[2] = csub(a0, b0);
    x[1] = cadd(a1, b1);
    x[3] = csub(a1, b1);
  } else if constexpr (RDX == 5) {
    const R c1 = (R)0.30901699437494742410, c2 = (R)-0.80901699437494742410;
    const R s1 = (R)0.95105651629515357212, s2 = (R)0.58778525229247312917;
    C a1 = cadd(x[1], x[4]), b1 = csub(x[1], x[4]);
    C a2 = cadd(x[2], x[3]), b2 = csub(x[2], x[3]);
    C x0 = x[0];
    C r1, r2, u1, u2;
    r1.x = x0.x + c1 * a1.x + c2 * a2.x;
    r1.y = x0.y + c1 * a1.y + c2 * a2.y;
    r2.x = x0.x + c2 * a1.x + c1 * a2.x;
    r2.y = x0.y + c2 * a1.y + c1 * a2.y;
    u1.x = s1 * b1.x + s2 * b2.x;
    u1.y = s1 * b1.y + s2 * b2.y;
    u2.x = s2 * b1.x - s1 * b2.x;
    u2.y = s2 * b1.y - s1 * b2.y;
    C i1 = cmul_si(u1, sign), i2 = cmul_si(u2, sign);
    x[0].x = x0.x + a1.x + a2.x;
    x[0].y = x0.y + a1.y + a2.y;
    x[1] = cadd(r1, i1);
    x[4] = csub(r1, i1);
    x[2] = cadd(r2, i2);
    x[3] = csub(r2, i2);
  } else if constexpr (RDX == 8) {
    const R r = (R)0.70710678118654752440;
    C e[4] = {x[0], x[2], x[4], x[6]};
    C o[4] = {x[1], x[3], x[5], x[7]};
    dft_small<4>(e, sign_d);
    dft_small<4>(o, sign_d);
    // o_t *= W8^t, W8 = exp(sign 2 pi i / 8)
    C t1, t3;
    t1.x = r * (o[1].x - sign * o[1].y);
    t1.y = r * (o[1].y + sign * o[1].x);
    t3.x = r * (-o[3].x - sign * o[3].y);
    t3.y = r * (-o[3].y + sign * o[3].x);
    o[1] = t1;
    o[2] = cmul_si(o[2], sign);
    o[3] = t3;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      x[t] = cadd(e[t], o[t]);
      x[t + 4] = csub(e[t], o[t]);
    }
  } else if constexpr (RDX == 9) {
    // 9 = 3 x 3: DFT3 over each residue class b of u = 3a + b, twiddle W9^{bc}, DFT3 over b.
    const double c1 = 0.76604444311897803520, s1 = 0.64278760968653932632;   // 2 pi / 9
    const double c2 = 0.17364817766693034885, s2 = 0.98480775301220805936;   // 4 pi / 9
    const double c4 = -0.93969262078590838405, s4 = 0.34202014332566873304;  // 8 pi / 9
    C y[3][3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      C t[3] = {x[b], x[b + 3], x[b + 6]};
      dft_small<3>(t, sign_d);
      y[b][0] = t[0];
      y[b][1] = t[1];
      y[b][2] = t[2];
    }
    const C w1 = mkc<C>(c1, sign_d * s1), w2 = mkc<C>(c2, sign_d * s2), w4 = mkc<C>(c4, sign_d * s4);
    y[1][1] = cmul(y[1][1], w1);
    y[1][2] = cmul(y[1][2], w2);
    y[2][1] = cmul(y[2][1], w2);
    y[2][2] = cmul(y[2][2], w4);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      C t[3] = {y[0][c], y[1][c], y[2][c]};
      dft_small<3>(t, sign_d);
      x[c] = t[0];
      x[c + 3] = t[1];
      x[c + 6] = t[2];
    }
  }
}

template <class C>
__device__ __forceinline__ void dft_any(C *x, int R, double sign) {
  switch (R) {
    case 2: dft_small<2>(x, sign); break;
    case 3: dft_small<3>(x, sign); break;
    case 4: dft_small<4>(x, sign); break;
    case 5: dft_small<5>(x, sign); break;
    case 8: dft_small<8>(x, sign); break;
    case 9: dft_small<9>(x, sign); break;
    default: break;
  }
}

// One in-place stage over `nlines` lines of length N stored in LDS.  Line i
// starts at base_i = b0[i] (or i * bstride when b0 == nullptr) with element
// stride es.  dif = true: butterfly then twiddle, sign +1; dif = false: conjugate
// twiddle then butterfly with sign -1 (the inverse-order stage).
template <class C>
__device__ __forceinline__ void fft_stage(C *P, int nlines, const int *lines, int lmul, int lmod, int lshift,
                                          int lstride, int es, int N, int R, int L, const C *tw, bool dif) {
  const int nb = N / R;
  const int B = R * L;
  const int tstep = N / B;
  const double sign = dif ? 1.0 : -1.0;
  for (int w = threadIdx.x; w < nlines * nb; w += blockDim.x) {
    const int line = w / nb;
    const int b = w - line * nb;
    const int blk = b / L;
    const int j = b - blk * L;
    int lb;
    if (lines) {
      int v = lines[line] - lshift;
      v %= lmod;
      if (v < 0) v += lmod;
      lb = v * lmul;
    } else {
      lb = line * lstride;
    }
    const int base = lb + (blk * B + j) * es;
    const int step = L * es;
    C x[9];
    for (int t = 0; t < R; ++t) x[t] = P[base + t * step];
    if (dif) {
      dft_any(x, R, sign);
      for (int t = 1; t < R; ++t) x[t] = cmul(x[t], tw[(j * t * tstep) % N]);
    } else {
      for (int t = 1; t < R; ++t) x[t] = cmulc(x[t], tw[(j * t * tstep) % N]);
      dft_any(x, R, sign);
    }
    for (int t = 0; t < R; ++t) P[base + t * step] = x[t];
  }
}

// Full transform of a set of lines: decimation in frequency (dif) or its reverse.
template <class C>
__device__ __forceinline__ void fft_lines(C *P, const C *tw, const Axis &a, int nlines, const int *lines, int lmul,
                                          int lmod, int lshift, int lstride, int es, bool dif) {
  if (dif) {
    for (int s = 0; s < a.nst; ++s) {
      fft_stage(P, nlines, lines, lmul, lmod, lshift, lstride, es, a.n, a.rad[s], a.span[s], tw, true);
      __syncthreads();
    }
  } else {
    for (int s = a.nst - 1; s >= 0; --s) {
      fft_stage(P, nlines, lines, lmul, lmod, lshift, lstride, es, a.n, a.rad[s], a.span[s], tw, false);
      __syncthreads();
    }
  }
}

__device__ __forceinline__ int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

template <class C>
__device__ __forceinline__ void plane_zero(C *P, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) P[i] = czero<C>();
}

__device__ __forceinline__ void basis_of(const KPair *kp, int k, int use_kq, int &e, int &g0x, int &g0y, int &g0z) {
  const KPair P = kp[k];
  if (use_kq) {
    e = P.ej;
    g0x = P.g0[0];
    g0y = P.g0[1];
    g0z = P.g0[2];
  } else {
    e = P.ek;
    g0x = g0y = g0z = 0;
  }
}

// ------------------------------------------------- compile-time transforms
// Radix order must match the host's factorization: at each step the first of
// 8, 9, 4, 2, 3, 5 that divides.
constexpr int crad(int n, int s) {
  for (int i = 0;; ++i) {
    const int r = (n % 8 == 0)   ? 8
                  : (n % 9 == 0) ? 9
                  : (n % 4 == 0) ? 4
                  : (n % 2 == 0) ? 2
                  : (n % 3 == 0) ? 3
                  : (n % 5 == 0) ? 5
                                 : 1;
    if (i == s || r == 1) return r;
    n /= r;
  }
}
constexpr int cnst(int n) {
  int k = 0;
  while (n > 1) {
    const int r = crad(n, 0);
    if (r == 1) return -1;
    n /= r;
    ++k;
  }
  return k;
}
constexpr int cspan(int n, int s) {
  int p = 1;
  for (int i = 0; i <= s; ++i) p *= crad(n, i);
  return n / p;
}

struct BaseList {  // line l starts at xs[l] * mul (xs already shifted and wrapped)
  const int *xs;
  int mul;
  __device__ __forceinline__ int operator()(int l) const { return xs[l] * mul; }
};
struct BaseAffine {  // line l starts at l * stride
  int stride;
  __device__ __forceinline__ int operator()(int l) const { return l * stride; }
};
// Batches of planes (np points each): line l is line l % n of plane l / n.
struct BaseListB {
  const int *xs;
  int mul, n, np;
  __device__ __forceinline__ int operator()(int l) const {
    const int p = l / n;
    return p * np + xs[l - p * n] * mul;
  }
};
template <int N, int NP>
struct BaseAffineB {
  __device__ __forceinline__ int operator()(int l) const {
    const int p = l / N;
    return p * NP + (l - p * N);
  }
};

// One radix-R stage over nlines lines. LF: consecutive threads take consecutive lines
// (for lines that are adjacent in LDS, strided elements), else consecutive butterflies
// of one line (for contiguous lines): either way neighbouring lanes hit neighbouring banks.
template <int N, int S, bool DIF, bool LF = false, class BaseF, class C>
__device__ __forceinline__ void cstage(C *__restrict__ P, const C *__restrict__ tw, int nlines, const BaseF &base,
                                       int es) {
  constexpr int R = crad(N, S), L = cspan(N, S), B = R * L, NB = N / R, TSTEP = N / B;
  const int total = nlines * NB;
  for (int w = threadIdx.x; w < total; w += blockDim.x) {
    const int line = LF ? w % nlines : w / NB;
    const int b = LF ? w / nlines : w - line * NB;
    const int blk = b / L;
    const int j = b - blk * L;
    const int o = base(line) + (blk * B + j) * es;
    C x[R];
#pragma unroll
    for (int t = 0; t < R; ++t) x[t] = P[o + t * L * es];
    if constexpr (DIF) {
      dft_small<R>(x, 1.0);
      if constexpr (L > 1) {
#pragma unroll
        for (int t = 1; t < R; ++t) x[t] = cmul(x[t], tw[j * t * TSTEP]);
      }
    } else {
      if constexpr (L > 1) {
#pragma unroll
        for (int t = 1; t < R; ++t) x[t] = cmulc(x[t], tw[j * t * TSTEP]);
      }
      dft_small<R>(x, -1.0);
    }
#pragma unroll
    for (int t = 0; t < R; ++t) P[o + t * L * es] = x[t];
  }
  __syncthreads();
}

template <int N, bool DIF, int I, bool LF = false, class BaseF, class C>
__device__ __forceinline__ void cfft(C *P, const C *tw, int nlines, const BaseF &base, int es) {
  constexpr int NS = cnst(N);
  static_assert(NS > 0, "FFT length must be a product of 2, 3 and 5");
  if constexpr (I < NS) {
    cstage<N, DIF ? I : NS - 1 - I, DIF, LF>(P, tw, nlines, base, es);
    cfft<N, DIF, I + 1, LF>(P, tw, nlines, base, es);
  }
}

// Stages I..E-1 of the transform (DIF order for DIF, reverse order otherwise).
template <int N, bool DIF, int I, int E, bool LF = false, class BaseF, class C>
__device__ __forceinline__ void cfft_range(C *P, const C *tw, int nlines, const BaseF &base, int es) {
  constexpr int NS = cnst(N);
  if constexpr (I < E) {
    cstage<N, DIF ? I : NS - 1 - I, DIF, LF>(P, tw, nlines, base, es);
    cfft_range<N, DIF, I + 1, E, LF>(P, tw, nlines, base, es);
  }
}

// The last forward (DIF) stage, a pointwise multiply by v and the first inverse stage in
// one pass: both stages have span 1 and visit the same R elements per work item, so the
// values stay in registers (the same operations as the three separate passes).
template <int N, bool LF, class BaseF, class C, class V>
__device__ __forceinline__ void cstage_mul(C *__restrict__ P, int nlines, const BaseF &base, int es,
                                           const V *__restrict__ v) {
  constexpr int NS = cnst(N);
  constexpr int R = crad(N, NS - 1), L = cspan(N, NS - 1), B = R * L, NB = N / R;
  static_assert(L == 1, "the last stage has span 1");
  const int total = nlines * NB;
  for (int w = threadIdx.x; w < total; w += blockDim.x) {
    const int line = LF ? w % nlines : w / NB;
    const int b = LF ? w / nlines : w - line * NB;
    const int o = base(line) + b * B * es;
    C x[R];
#pragma unroll
    for (int t = 0; t < R; ++t) x[t] = P[o + t * es];
    dft_small<R>(x, 1.0);
#pragma unroll
    for (int t = 0; t < R; ++t) x[t] = cscale(x[t], v[o + t * es]);
    dft_small<R>(x, -1.0);
#pragma unroll
    for (int t = 0; t < R; ++t) P[o + t * es] = x[t];
  }
  __syncthreads();
}

// Per-block plane context: LDS tables and the transforms of one xy plane.
// N1 = N2 = 0 selects the runtime-size path; C is double2 (FP64) or float2 (FP32).
template <class C>
__device__ __forceinline__ const C *axis_tw(const Axis &a);
template <>
__device__ __forceinline__ const double2 *axis_tw<double2>(const Axis &a) {
  return a.tw;
}
template <>
__device__ __forceinline__ const float2 *axis_tw<float2>(const Axis &a) {
  return a.tw32;
}

// TG: the twiddle tables are read from global memory (cached) instead of LDS copies,
// which leaves more of the LDS for planes of other workgroups.
template <int N1, int N2, class C = double2, int PB = 1, bool TG = false>
struct PlaneCtx {
  static_assert(PB == 1 || (N1 > 0 && N2 > 0), "plane batches need compile-time plane sizes");
  const Plane &pl;
  C *P;            // [PB][n1*n2]
  const C *twx;    // [n1] (LDS copy, or the global table when TG)
  const C *twy;    // [n2]
  int *xs;         // [n1] active x columns, shifted and wrapped
  int nxa;
  __device__ __forceinline__ int n1() const { return N1 > 0 ? N1 : pl.n1; }
  __device__ __forceinline__ int n2() const { return N2 > 0 ? N2 : pl.n2; }
  __device__ __forceinline__ int np() const { return n1() * n2(); }
  __device__ __forceinline__ PlaneCtx(const Plane &p, void *lds) : pl(p) {
    P = reinterpret_cast<C *>(lds);
    nxa = 0;
    const C *tx = axis_tw<C>(pl.ax), *ty = axis_tw<C>(pl.ay);
    if constexpr (TG) {
      twx = tx;
      twy = ty;
      xs = reinterpret_cast<int *>(P + PB * np());
    } else {
      C *lx = P + PB * np();
      C *ly = lx + n1();
      for (int i = threadIdx.x; i < n1(); i += blockDim.x) lx[i] = tx[i];
      for (int i = threadIdx.x; i < n2(); i += blockDim.x) ly[i] = ty[i];
      twx = lx;
      twy = ly;
      xs = reinterpret_cast<int *>(ly + n2());
    }
  }
  // active x list of a stick set shifted by g0x (call from every thread; ends with a barrier)
  __device__ __forceinline__ void set_active(const int *xa, int n, int g0x) {
    nxa = n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) xs[i] = wrap(xa[i] - g0x, n1());
    __syncthreads();
  }
  __device__ __forceinline__ void set_all_x() {
    nxa = n1();
    for (int i = threadIdx.x; i < n1(); i += blockDim.x) xs[i] = i;
    __syncthreads();
  }
  template <bool DIF>
  __device__ __forceinline__ void y_lines() {  // lines at the listed x, contiguous, length N2
    if constexpr (PB > 1) {
      cfft<N2, DIF, 0>(P, twy, nxa * PB, BaseListB{xs, N2, nxa, N1 * N2}, 1);
    } else if constexpr (N2 > 0) {
      cfft<N2, DIF, 0>(P, twy, nxa, BaseList{xs, N2}, 1);
    } else {
      fft_lines(P, twy, pl.ay, nxa, xs, pl.n2, pl.n1, 0, 0, 1, DIF);
    }
  }
  template <bool DIF>
  __device__ __forceinline__ void x_lines() {  // every y, stride N2, length N1
    if constexpr (PB > 1) {
      cfft<N1, DIF, 0, true>(P, twx, N2 * PB, BaseAffineB<N2, N1 * N2>{}, N2);
    } else if constexpr (N1 > 0) {
      cfft<N1, DIF, 0, true>(P, twx, N2, BaseAffine{1}, N2);
    } else {
      fft_lines(P, twx, pl.ax, pl.n2, nullptr, 0, 1, 0, 1, pl.n2, DIF);
    }
  }
  // x_lines<true>, multiply by v (same layout as the plane batch), x_lines<false>
  template <class V>
  __device__ __forceinline__ void x_round_trip_mul(const V *__restrict__ v) {
    if constexpr (N1 > 0) {
      constexpr int NS = cnst(N1);
      if constexpr (PB > 1) {
        const BaseAffineB<N2, N1 * N2> base{};
        cfft_range<N1, true, 0, NS - 1, true>(P, twx, N2 * PB, base, N2);
        cstage_mul<N1, true>(P, N2 * PB, base, N2, v);
        cfft_range<N1, false, 1, NS, true>(P, twx, N2 * PB, base, N2);
      } else {
        const BaseAffine base{1};
        cfft_range<N1, true, 0, NS - 1, true>(P, twx, N2, base, N2);
        cstage_mul<N1, true>(P, N2, base, N2, v);
        cfft_range<N1, false, 1, NS, true>(P, twx, N2, base, N2);
      }
    } else {
      x_lines<true>();
      for (int i = threadIdx.x; i < np(); i += blockDim.x) P[i] = cscale(P[i], v[i]);
      __syncthreads();
      x_lines<false>();
    }
  }
  __device__ __forceinline__ int pos(int x, int y, int g0x, int g0y) const {
    return wrap(x - g0x, n1()) * n2() + wrap(y - g0y, n2());
  }
};

int plane_lds_t(const Plane &pl, int csize = (int)sizeof(double2), int pb = 1, bool tw_global = false) {
  return pb * pl.n1 * pl.n2 * csize + (tw_global ? 0 : (pl.n1 + pl.n2) * csize) + pl.n1 * (int)sizeof(int);
}

// ----------------------------------------------------------------- kernels

template <class C>
using RealOf = decltype(C{}.x);

template <int N3, class C>
__global__ void __launch_bounds__(kThreads) k_stick_inv(Sticks sk, const KPair *kp, int use_kq, int nb,
                                                        const C *__restrict__ X, int ld, C *__restrict__ S,
                                                        int ns_pad, int n3_rt, const C *__restrict__ tw3,
                                                        const int *active) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *smem = reinterpret_cast<C *>(smem_raw);
  const int n3 = N3 > 0 ? N3 : n3_rt;
  const int item = blockIdx.y;
  if (active && !active[item]) return;
  const int k = item / nb;
  int e, g0x, g0y, g0z;
  basis_of(kp, k, use_kq, e, g0x, g0y, g0z);
  const EntryDev E = sk.ent[e];
  const int s0 = blockIdx.x * kStickChunk;
  if (s0 >= E.ns) return;
  const int s1 = min(s0 + kStickChunk, E.ns);
  const int *sstart = sk.sstart + E.st_off;
  const int *slen = sk.slen + E.st_off;
  const int p0 = sstart[s0];
  const int p1 = sstart[s1 - 1] + slen[s1 - 1];
  C *tw = smem;          // [n3]
  C *c = smem + n3;      // [p1 - p0]
  int *zi = reinterpret_cast<int *>(c + (p1 - p0));
  for (int i = threadIdx.x; i < n3; i += blockDim.x) tw[i] = tw3[i];
  const C *x = X + (size_t)item * ld;
  for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    c[p - p0] = x[p];
    zi[p - p0] = wrap(sk.iz[E.pw_off + p] - g0z, n3);
  }
  __syncthreads();
  const int nsc = s1 - s0;
  C *out = S + (size_t)item * n3 * ns_pad;
  for (int idx = threadIdx.x; idx < nsc * n3; idx += blockDim.x) {
    const int z = idx / nsc;
    const int s = s0 + (idx - z * nsc);
    const int a = sstart[s] - p0;
    const int len = slen[s];
    C acc = czero<C>();
    for (int t = 0; t < len; ++t) acc = cadd(acc, cmul(c[a + t], tw[(zi[a + t] * z) % n3]));
    out[(size_t)z * ns_pad + s] = acc;
  }
}

template <int N3, class C>
__global__ void __launch_bounds__(kThreads) k_stick_fwd(Sticks sk, const KPair *kp, int use_kq, int nb,
                                                        const C *__restrict__ S, int ns_pad, int n3_rt,
                                                        const C *__restrict__ tw3, double scale,
                                                        C *__restrict__ Y, int ld, int mode,
                                                        const double *__restrict__ kin,
                                                        const double *__restrict__ eps,
                                                        const C *__restrict__ X, int eps_stride,
                                                        const int *active) {
  using R = RealOf<C>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *smem = reinterpret_cast<C *>(smem_raw);
  const int n3 = N3 > 0 ? N3 : n3_rt;
  const int item = blockIdx.y;
  if (active && !active[item]) return;
  const int k = item / nb;
  const int v = item - k * nb;
  int e, g0x, g0y, g0z;
  basis_of(kp, k, use_kq, e, g0x, g0y, g0z);
  const EntryDev E = sk.ent[e];
  const int s0 = blockIdx.x * kStickChunk;
  if (s0 >= E.ns) return;
  const int s1 = min(s0 + kStickChunk, E.ns);
  const int nsc = s1 - s0;
  const int *sstart = sk.sstart + E.st_off;
  const int *slen = sk.slen + E.st_off;
  const int p0 = sstart[s0];
  const int p1 = sstart[s1 - 1] + slen[s1 - 1];
  C *tw = smem;                                       // [n3]
  C *sl = smem + n3;                                  // [n3][nsc]
  int *own = reinterpret_cast<int *>(sl + n3 * nsc);  // [p1-p0] stick of each plane wave
  for (int i = threadIdx.x; i < n3; i += blockDim.x) tw[i] = tw3[i];
  if (S) {
    const C *in = S + (size_t)item * n3 * ns_pad;
    for (int idx = threadIdx.x; idx < nsc * n3; idx += blockDim.x) {
      const int z = idx / nsc;
      const int s = idx - z * nsc;
      sl[idx] = in[(size_t)z * ns_pad + s0 + s];
    }
  }
  for (int s = s0 + threadIdx.x; s < s1; s += blockDim.x)
    for (int t = 0; t < slen[s]; ++t) own[sstart[s] - p0 + t] = s - s0;
  __syncthreads();
  C *y = Y + (size_t)item * ld;
  const C *x = X ? X + (size_t)item * ld : nullptr;
  const double ev = eps ? eps[(size_t)k * eps_stride + v] : 0.0;
  for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    C acc = czero<C>();
    if (S) {
      const int s = own[p - p0];
      const int zz = wrap(sk.iz[E.pw_off + p] - g0z, n3);
      int ix = 0;
      for (int z = 0; z < n3; ++z) {
        acc = cadd(acc, cmulc(sl[z * nsc + s], tw[ix]));
        ix += zz;
        if (ix >= n3) ix -= n3;
      }
      acc = cscale(acc, scale);
    }
    if (mode == 0) {
      const C xv = x[p];
      const R d = (R)(kin[E.pw_off + p] - ev);
      acc.x += d * xv.x;
      acc.y += d * xv.y;
    }
    y[p] = acc;
  }
}

// The z transforms with one thread per stick: the stick's N3 values stay in registers
// while its plane waves are visited once.  The sums run over the same terms in the same
// order as in k_stick_inv / k_stick_fwd, so the results are the same.
template <int N3, class C>
__global__ void __launch_bounds__(kThreads) k_stick_inv_s(Sticks sk, const KPair *kp, int use_kq, int nb,
                                                          const C *__restrict__ X, int ld, C *__restrict__ S,
                                                          int ns_pad, const C *__restrict__ tw3, const int *active) {
  __shared__ C tw[N3];
  const int item = blockIdx.y;
  if (active && !active[item]) return;
  const int k = item / nb;
  int e, g0x, g0y, g0z;
  basis_of(kp, k, use_kq, e, g0x, g0y, g0z);
  const EntryDev E = sk.ent[e];
  if ((int)(blockIdx.x * blockDim.x) >= E.ns) return;
  for (int i = threadIdx.x; i < N3; i += blockDim.x) tw[i] = tw3[i];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= E.ns) return;
  const int a = sk.sstart[E.st_off + s], len = sk.slen[E.st_off + s];
  const C *x = X + (size_t)item * ld + a;
  const int *izp = sk.iz + E.pw_off + a;
  C acc[N3];
#pragma unroll
  for (int z = 0; z < N3; ++z) acc[z] = czero<C>();
  for (int t = 0; t < len; ++t) {
    const C c = x[t];
    const int zi = wrap(izp[t] - g0z, N3);
    int ix = 0;
#pragma unroll
    for (int z = 0; z < N3; ++z) {
      acc[z] = cadd(acc[z], cmul(c, tw[ix]));
      ix += zi;
      if (ix >= N3) ix -= N3;
    }
  }
  C *out = S + (size_t)item * N3 * ns_pad + s;
#pragma unroll
  for (int z = 0; z < N3; ++z) out[(size_t)z * ns_pad] = acc[z];
}

template <int N3, class C>
__global__ void __launch_bounds__(kThreads) k_stick_fwd_s(Sticks sk, const KPair *kp, int use_kq, int nb,
                                                          const C *__restrict__ S, int ns_pad,
                                                          const C *__restrict__ tw3, double scale,
                                                          C *__restrict__ Y, int ld, int mode,
                                                          const double *__restrict__ kin,
                                                          const double *__restrict__ eps,
                                                          const C *__restrict__ X, int eps_stride,
                                                          const int *active) {
  using R = RealOf<C>;
  __shared__ C tw[N3];
  const int item = blockIdx.y;
  if (active && !active[item]) return;
  const int k = item / nb;
  const int v = item - k * nb;
  int e, g0x, g0y, g0z;
  basis_of(kp, k, use_kq, e, g0x, g0y, g0z);
  const EntryDev E = sk.ent[e];
  if ((int)(blockIdx.x * blockDim.x) >= E.ns) return;
  for (int i = threadIdx.x; i < N3; i += blockDim.x) tw[i] = tw3[i];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= E.ns) return;
  const int a = sk.sstart[E.st_off + s], len = sk.slen[E.st_off + s];
  C sv[N3];
  if (S) {
    const C *in = S + (size_t)item * N3 * ns_pad + s;
#pragma unroll
    for (int z = 0; z < N3; ++z) sv[z] = in[(size_t)z * ns_pad];
  }
  C *y = Y + (size_t)item * ld;
  const C *x = X ? X + (size_t)item * ld : nullptr;
  const double ev = eps ? eps[(size_t)k * eps_stride + v] : 0.0;
  for (int t = 0; t < len; ++t) {
    const int p = a + t;
    C acc = czero<C>();
    if (S) {
      const int zz = wrap(sk.iz[E.pw_off + p] - g0z, N3);
      int ix = 0;
#pragma unroll
      for (int z = 0; z < N3; ++z) {
        acc = cadd(acc, cmulc(sv[z], tw[ix]));
        ix += zz;
        if (ix >= N3) ix -= N3;
      }
      acc = cscale(acc, scale);
    }
    if (mode == 0) {
      const C xv = x[p];
      const R d = (R)(kin[E.pw_off + p] - ev);
      acc.x += d * xv.x;
      acc.y += d * xv.y;
    }
    y[p] = acc;
  }
}

// The thread-per-stick transforms with the plane waves of the workgroup's sticks (a
// contiguous range) staged through LDS, so that global memory is read (inverse) or written
// (forward) in coalesced rows instead of one stick per lane; the sums are those of
// k_stick_inv_s / k_stick_fwd_s, term by term.
template <int N3, class C>
__global__ void __launch_bounds__(kThreads) k_stick_inv_sl(Sticks sk, const KPair *kp, int use_kq, int nb,
                                                           const C *__restrict__ X, int ld, C *__restrict__ S,
                                                           int ns_pad, const C *__restrict__ tw3, const int *active) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *tw = reinterpret_cast<C *>(smem_raw);  // [N3]
  C *cv = tw + N3;                          // [p1 - p0] coefficients
  const int item = blockIdx.y;
  if (active && !active[item]) return;
  const int k = item / nb;
  int e, g0x, g0y, g0z;
  basis_of(kp, k, use_kq, e, g0x, g0y, g0z);
  const EntryDev E = sk.ent[e];
  const int s0 = blockIdx.x * kThreads;
  if (s0 >= E.ns) return;
  const int s1 = min(s0 + kThreads, E.ns);
  const int *sstart = sk.sstart + E.st_off, *slen = sk.slen + E.st_off;
  const int p0 = sstart[s0], p1 = sstart[s1 - 1] + slen[s1 - 1];
  int *zi = reinterpret_cast<int *>(cv + (p1 - p0));  // [p1 - p0] z index (shifted, wrapped)
  for (int i = threadIdx.x; i < N3; i += kThreads) tw[i] = tw3[i];
  const C *x = X + (size_t)item * ld;
  for (int p = p0 + threadIdx.x; p < p1; p += kThreads) {
    cv[p - p0] = x[p];
    zi[p - p0] = wrap(sk.iz[E.pw_off + p] - g0z, N3);
  }
  __syncthreads();
  const int s = s0 + threadIdx.x;
  if (s >= s1) return;
  const int a = sstart[s] - p0, len = slen[s];
  C acc[N3];
#pragma unroll
  for (int z = 0; z < N3; ++z) acc[z] = czero<C>();
  for (int t = 0; t < len; ++t) {
    const C c = cv[a + t];
    const int zz = zi[a + t];
    int ix = 0;
#pragma unroll
    for (int z = 0; z < N3; ++z) {
      acc[z] = cadd(acc[z], cmul(c, tw[ix]));
      ix += zz;
      if (ix >= N3) ix -= N3;
    }
  }
  C *out = S + (size_t)item * N3 * ns_pad + s;
#pragma unroll
  for (int z = 0; z < N3; ++z) out[(size_t)z * ns_pad] = acc[z];
}

template <int N3, class C>
__global__ void __launch_bounds__(kThreads) k_stick_fwd_sl(Sticks sk, const KPair *kp, int use_kq, int nb,
                                                           const C *__restrict__ S, int ns_pad,
                                                           const C *__restrict__ tw3, double scale,
                                                           C *__restrict__ Y, int ld, int mode,
                                                           const double *__restrict__ kin,
                                                           const double *__restrict__ eps,
                                                           const C *__restrict__ X, int eps_stride,
                                                           const int *active) {
  using R = RealOf<C>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *tw = reinterpret_cast<C *>(smem_raw);  // [N3]
  C *yb = tw + N3;                          // [p1 - p0] stick sums of this workgroup's plane waves
  const int item = blockIdx.y;
  if (active && !active[item]) return;
  const int k = item / nb;
  const int v = item - k * nb;
  int e, g0x, g0y, g0z;
  basis_of(kp, k, use_kq, e, g0x, g0y, g0z);
  const EntryDev E = sk.ent[e];
  const int s0 = blockIdx.x * kThreads;
  if (s0 >= E.ns) return;
  const int s1 = min(s0 + kThreads, E.ns);
  const int *sstart = sk.sstart + E.st_off, *slen = sk.slen + E.st_off;
  const int p0 = sstart[s0], p1 = sstart[s1 - 1] + slen[s1 - 1];
  for (int i = threadIdx.x; i < N3; i += kThreads) tw[i] = tw3[i];
  __syncthreads();
  const int s = s0 + threadIdx.x;
  if (s < s1) {
    const int a = sstart[s], len = slen[s];
    if (S) {
      C sv[N3];
      const C *in = S + (size_t)item * N3 * ns_pad + s;
#pragma unroll
      for (int z = 0; z < N3; ++z) sv[z] = in[(size_t)z * ns_pad];
      for (int t = 0; t < len; ++t) {
        const int p = a + t;
        const int zz = wrap(sk.iz[E.pw_off + p] - g0z, N3);
        C acc = czero<C>();
        int ix = 0;
#pragma unroll
        for (int z = 0; z < N3; ++z) {
          acc = cadd(acc, cmulc(sv[z], tw[ix]));
          ix += zz;
          if (ix >= N3) ix -= N3;
        }
        yb[p - p0] = cscale(acc, scale);
      }
    } else {
      for (int t = 0; t < len; ++t) yb[a + t - p0] = czero<C>();
    }
  }
  __syncthreads();
  C *y = Y + (size_t)item * ld;
  const C *x = X ? X + (size_t)item * ld : nullptr;
  const double ev = eps ? eps[(size_t)k * eps_stride + v] : 0.0;
  for (int p = p0 + threadIdx.x; p < p1; p += kThreads) {
    C acc = yb[p - p0];
    if (mode == 0) {
      const C xv = x[p];
      const R d = (R)(kin[E.pw_off + p] - ev);
      acc.x += d * xv.x;
      acc.y += d * xv.y;
    }
    y[p] = acc;
  }
}

template <int N1, int N2, class C>
__global__ void __launch_bounds__(kThreads) k_plane_vloc(Plane pl, Sticks sk, const KPair *kp, int use_kq, int nb,
                                                         const C *__restrict__ Sin, C *__restrict__ Sout,
                                                         int ns_pad, const RealOf<C> *__restrict__ vp,
                                                         const int *active) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int item = blockIdx.y;
  if (active && !active[item]) return;
  PlaneCtx<N1, N2, C> pc(pl, lds);
  const int z = blockIdx.x;
  const int k = item / nb;
  int e, g0x, g0y, g0z;
  basis_of(kp, k, use_kq, e, g0x, g0y, g0z);
  const EntryDev E = sk.ent[e];
  const int np = pc.np();
  C *P = pc.P;
  plane_zero(P, np);
  pc.set_active(sk.xa + E.xa_off, E.nxa, g0x);
  const int *sx = sk.sx + E.st_off;
  const int *sy = sk.sy + E.st_off;
  const size_t so = ((size_t)item * pl.n3 + z) * ns_pad;
  for (int s = threadIdx.x; s < E.ns; s += blockDim.x) P[pc.pos(sx[s], sy[s], g0x, g0y)] = Sin[so + s];
  __syncthreads();
  pc.template y_lines<true>();
  pc.x_round_trip_mul(vp + ((size_t)kp[k].spin * pl.n3 + z) * np);
  pc.template y_lines<false>();
  for (int s = threadIdx.x; s < E.ns; s += blockDim.x) Sout[so + s] = P[pc.pos(sx[s], sy[s], g0x, g0y)];
}

// The same round trip for PB consecutive z planes of one item per workgroup of NT threads
// (the transform stages then run over PB times as many lines per barrier).
template <int N1, int N2, class C, int PB, int NT, bool TG = false>
__global__ void __launch_bounds__(NT) k_plane_vloc_b(Plane pl, Sticks sk, const KPair *kp, int use_kq, int nb,
                                                     const C *__restrict__ Sin, C *__restrict__ Sout, int ns_pad,
                                                     const RealOf<C> *__restrict__ vp, const int *active) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int item = blockIdx.y;
  if (active && !active[item]) return;
  PlaneCtx<N1, N2, C, PB, TG> pc(pl, lds);
  constexpr int np = N1 * N2;
  const int z0 = blockIdx.x * PB;
  const int k = item / nb;
  int e, g0x, g0y, g0z;
  basis_of(kp, k, use_kq, e, g0x, g0y, g0z);
  const EntryDev E = sk.ent[e];
  C *P = pc.P;
  plane_zero(P, PB * np);
  pc.set_active(sk.xa + E.xa_off, E.nxa, g0x);
  const int *sx = sk.sx + E.st_off;
  const int *sy = sk.sy + E.st_off;
  const size_t so = ((size_t)item * pl.n3 + z0) * ns_pad;
  for (int w = threadIdx.x; w < PB * E.ns; w += NT) {
    const int p = w / E.ns, s = w - p * E.ns;
    P[p * np + pc.pos(sx[s], sy[s], g0x, g0y)] = Sin[so + (size_t)p * ns_pad + s];
  }
  __syncthreads();
  pc.template y_lines<true>();
  pc.x_round_trip_mul(vp + ((size_t)kp[k].spin * pl.n3 + z0) * np);
  pc.template y_lines<false>();
  for (int w = threadIdx.x; w < PB * E.ns; w += NT) {
    const int p = w / E.ns, s = w - p * E.ns;
    Sout[so + (size_t)p * ns_pad + s] = P[p * np + pc.pos(sx[s], sy[s], g0x, g0y)];
  }
}

// ------------------------------------------- register-resident plane round trip (FP32)
// A thread holds a whole line in registers and runs every radix stage of it there, with the
// same butterflies, twiddles and order of operations as the LDS stages above (so the
// results are those of the LDS variants); LDS only carries the two transposes (y columns ->
// x rows -> y columns).  An x line longer than 72 points whose last radix is 2 is split over
// two neighbouring lanes by parity: each lane runs the stages before the last on its 72
// points, and the last radix-2 stage (fused with the multiply by V and the first inverse
// stage) exchanges values with the partner lane through DPP.

// The partner lane's value (lane ^ 1, DPP quad permutation [1, 0, 3, 2]).
__device__ __forceinline__ float lane_xor1(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// Stage S of a length-N line held whole in x[0..N): DIF (butterfly, then twiddle) or the
// reverse-order inverse stage (conjugate twiddle, then butterfly).
template <int N, int S, bool DIF, class C>
__device__ __forceinline__ void rstage(C *x, const C *__restrict__ tw) {
  constexpr int R = crad(N, S), L = cspan(N, S), B = R * L, TSTEP = N / B;
#pragma unroll
  for (int blk = 0; blk < N / B; ++blk)
#pragma unroll
    for (int j = 0; j < L; ++j) {
      C y[R];
#pragma unroll
      for (int t = 0; t < R; ++t) y[t] = x[blk * B + j + t * L];
      if constexpr (DIF) {
        dft_small<R>(y, 1.0);
        if constexpr (L > 1) {
#pragma unroll
          for (int t = 1; t < R; ++t) y[t] = cmul(y[t], tw[j * t * TSTEP]);
        }
      } else {
        if constexpr (L > 1) {
#pragma unroll
          for (int t = 1; t < R; ++t) y[t] = cmulc(y[t], tw[j * t * TSTEP]);
        }
        dft_small<R>(y, -1.0);
      }
#pragma unroll
      for (int t = 0; t < R; ++t) x[blk * B + j + t * L] = y[t];
      __builtin_amdgcn_sched_barrier(0);  // one butterfly at a time: bounded register use
    }
}

// Stages I..E-1 in DIF order (DIF) or stages E-1..I in inverse order.
template <int N, int I, int E, bool DIF, class C>
__device__ __forceinline__ void rstages(C *x, const C *__restrict__ tw) {
  if constexpr (I < E) {
    if constexpr (DIF) {
      rstage<N, I, true>(x, tw);
      rstages<N, I + 1, E, true>(x, tw);
    } else {
      rstage<N, E - 1, false>(x, tw);
      rstages<N, I, E - 1, false>(x, tw);
    }
  }
}

// Stage S (span >= 2, even) of a length-N line split by parity: this lane holds
// h[u] = line[2u + par], u < N/2.
template <int N, int S, bool DIF, class C>
__device__ __forceinline__ void rstage_half(C *h, const C *__restrict__ tw, int par) {
  constexpr int R = crad(N, S), L = cspan(N, S), B = R * L, TSTEP = N / B;
  static_assert(L % 2 == 0, "a split stage needs an even span");
#pragma unroll
  for (int blk = 0; blk < N / B; ++blk)
#pragma unroll
    for (int jh = 0; jh < L / 2; ++jh) {
      C y[R];
#pragma unroll
      for (int t = 0; t < R; ++t) y[t] = h[blk * (B / 2) + jh + t * (L / 2)];
      // j = 2 jh + par: the twiddle of either parity, chosen per lane
      auto twid = [&](int t) {
        const C a = tw[(2 * jh) * t * TSTEP], b = tw[(2 * jh + 1) * t * TSTEP];
        return par ? b : a;
      };
      if constexpr (DIF) {
        dft_small<R>(y, 1.0);
#pragma unroll
        for (int t = 1; t < R; ++t) y[t] = cmul(y[t], twid(t));
      } else {
#pragma unroll
        for (int t = 1; t < R; ++t) y[t] = cmulc(y[t], twid(t));
        dft_small<R>(y, -1.0);
      }
#pragma unroll
      for (int t = 0; t < R; ++t) h[blk * (B / 2) + jh + t * (L / 2)] = y[t];
      // keep each butterfly's per-lane twiddles next to it (hoisted, they fill the registers)
      __builtin_amdgcn_sched_barrier(0);
    }
}

template <int N, int I, int E, bool DIF, class C>
__device__ __forceinline__ void rstages_half(C *h, const C *__restrict__ tw, int par) {
  if constexpr (I < E) {
    if constexpr (DIF) {
      rstage_half<N, I, true>(h, tw, par);
      rstages_half<N, I + 1, E, true>(h, tw, par);
    } else {
      rstage_half<N, E - 1, false>(h, tw, par);
      rstages_half<N, I, E - 1, false>(h, tw, par);
    }
  }
}

// Register-resident variants: the window [0, W) u [N - W, N) of x columns and y rows that
// may hold sphere points (even W near N / 3; a grid of at least four times the sphere's
// radius keeps the sphere inside it), and the LDS header (the active column list).
__host__ __device__ constexpr int reg_win(int n) { return ((n + 5) / 6) * 2; }
__host__ __device__ constexpr int reg_lds_header_c(int n1) { return ((n1 * 4 + 15) / 16) * 16; }
__host__ __device__ constexpr int reg_cols(int n1) { return 2 * reg_win(n1) < n1 ? 2 * reg_win(n1) : n1; }

// Rows of the plane (x lines) handled by one lane, or by a lane pair for long lines.
template <int N1>
struct RowSplit {
  static constexpr int NS = cnst(N1);
  static constexpr int RS = (N1 > 72 && crad(N1, NS - 1) == 2) ? 2 : 1;
  static constexpr int H = N1 / RS;
};

// Workgroup of NT threads: npb consecutive z planes of one band item (set by the launcher
// so that the lines fill the threads).  Only the x columns and y rows of the window
// [0, W) u [N - W, N) (reg_win) can hold sphere points (the launcher checks every entry's
// Miller range, shifted by the k+q pairs' g0, against it), so LDS keeps the planes compacted
// to the NC = 2 WX window columns, [plane][NC][N2 | 1] (an odd row stride keeps the column
// and the row accesses free of bank conflicts), after the list of active columns.  Outside
// the window the row and column inputs are zeros known at compile time (not loaded) and
// their outputs are not needed (not computed back).
template <int N1, int N2, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) k_plane_vloc_r(Plane pl, Sticks sk, const KPair *kp, int use_kq, int nb,
                                                     int npb, const float2 *__restrict__ Sin,
                                                     float2 *__restrict__ Sout, int ns_pad,
                                                     const float *__restrict__ vp, const int *active) {
  using C = float2;
  constexpr int N2S = N2 | 1;
  constexpr int WX = reg_win(N1), WY = reg_win(N2);
  constexpr int NC = 2 * WX < N1 ? 2 * WX : N1, XOFF = N1 - NC;  // window column of x >= N1 - WX: x - XOFF
  constexpr bool YCUT = 2 * WY < N2;
  constexpr int PS = NC * N2S;
  constexpr int RS = RowSplit<N1>::RS, H = RowSplit<N1>::H;
  constexpr int NS1 = cnst(N1), NS2 = cnst(N2);
  static_assert(H <= 72 && N2 <= 72, "line too long for registers");
  static_assert(RS == 1 || (WX % 2 == 0 && XOFF % 2 == 0), "a split row needs an even window");
  extern __shared__ __align__(16) unsigned char lds[];
  int *colc = reinterpret_cast<int *>(lds);  // [NC]: window column of each active x
  C *P = reinterpret_cast<C *>(lds + reg_lds_header_c(N1));
  const int item = blockIdx.y;
  if (active && !active[item]) return;
  const int k = item / nb;
  int e, g0x, g0y, g0z;
  basis_of(kp, k, use_kq, e, g0x, g0y, g0z);
  const EntryDev E = sk.ent[e];
  const int nxa = min(E.nxa, NC), ns = E.ns;
  const int z0 = blockIdx.x * npb;
  const int npl = min(npb, pl.n3 - z0);
  const C *twx = pl.ax.tw32, *twy = pl.ay.tw32;
  // window column of grid x (x in the window; -1 outside, which the launcher rules out)
  auto wcol = [](int x) { return x < WX ? x : (x >= N1 - WX ? x - XOFF : -1); };
  {
    float4 *P4 = reinterpret_cast<float4 *>(P);  // PS * npl float2, an even count when npl is even
    const int n4 = (npl * PS) / 2;
    for (int i = threadIdx.x; i < n4; i += NT) P4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    if ((npl * PS) & 1)
      if (threadIdx.x == 0) P[npl * PS - 1] = czero<C>();
  }
  const int *xa = sk.xa + E.xa_off;
  for (int i = threadIdx.x; i < nxa; i += NT) colc[i] = wcol(wrap(xa[i] - g0x, N1));
  __syncthreads();
  const int *sx = sk.sx + E.st_off;
  const int *sy = sk.sy + E.st_off;
  const size_t so = ((size_t)item * pl.n3 + z0) * ns_pad;
  for (int w = threadIdx.x; w < npl * ns; w += NT) {
    const int p = w / ns, s = w - p * ns;
    const int c = wcol(wrap(sx[s] - g0x, N1));
    if (c >= 0) P[p * PS + c * N2S + wrap(sy[s] - g0y, N2)] = Sin[so + (size_t)p * ns_pad + s];
  }
  __syncthreads();
  // y columns, forward (DIF): natural order in (zeros outside the y window), digit-reversed out
  for (int w = threadIdx.x; w < npl * nxa; w += NT) {
    const int p = w / nxa;
    const int c = colc[w - p * nxa];
    if (c < 0) continue;
    C *col = P + p * PS + c * N2S;
    C y[N2];
#pragma unroll
    for (int i = 0; i < N2; ++i) y[i] = (!YCUT || i < WY || i >= N2 - WY) ? col[i] : czero<C>();
    rstages<N2, 0, NS2, true>(y, twy);
#pragma unroll
    for (int i = 0; i < N2; ++i) col[i] = y[i];
  }
  __syncthreads();
  // x rows: forward, times V (digit-reversed x and y), inverse.  This lane holds the points
  // x = RS u + par of row r: window columns are read and written at fixed offsets, the
  // rest are zeros in and unused out.
  const float *vz = vp + ((size_t)kp[k].spin * pl.n3 + z0) * (N1 * N2);
  for (int w = threadIdx.x; w < npl * N2 * RS; w += NT) {
    const int p = w / (N2 * RS), rem = w - p * (N2 * RS);
    const int r = rem / RS, par = rem - r * RS;
    C *row = P + p * PS + par * N2S + r;
    const float *v = vz + (size_t)p * (N1 * N2) + r;
    C h[H];
#pragma unroll
    for (int u = 0; u < H; ++u) {
      const int x0 = RS * u;  // x = x0 + par; the window test is the same for both parities
      h[u] = x0 < WX ? row[x0 * N2S] : (x0 >= N1 - WX ? row[(x0 - XOFF) * N2S] : czero<C>());
    }
    // V is read in groups of G values, one group ahead of its use: without the schedule
    // barriers the compiler issues all H loads at once and the row no longer fits the
    // register file
    constexpr int G = RS == 1 ? crad(N1, NS1 - 1) : 8;
    static_assert(H % G == 0, "V groups");
    float vb[G], vn[G];
#pragma unroll
    for (int t = 0; t < G; ++t) vb[t] = v[(RS * t + par) * N2];
    if constexpr (RS == 1) {
      rstages<N1, 0, NS1 - 1, true>(h, twx);
      // last forward stage, times V, first inverse stage (span 1: within the thread)
#pragma unroll
      for (int b = 0; b < N1 / G; ++b) {
        if (b + 1 < N1 / G) {
#pragma unroll
          for (int t = 0; t < G; ++t) vn[t] = v[((b + 1) * G + t) * N2];
        }
        __builtin_amdgcn_sched_barrier(0);
        C y[G];
#pragma unroll
        for (int t = 0; t < G; ++t) y[t] = h[b * G + t];
        dft_small<G>(y, 1.0);
#pragma unroll
        for (int t = 0; t < G; ++t) y[t] = cscale(y[t], vb[t]);
        dft_small<G>(y, -1.0);
#pragma unroll
        for (int t = 0; t < G; ++t) h[b * G + t] = y[t];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < G; ++t) vb[t] = vn[t];
      }
      rstages<N1, 0, NS1 - 1, false>(h, twx);
    } else {
      rstages_half<N1, 0, NS1 - 1, true>(h, twx, par);
      // last stage: radix 2 over the pair (2u, 2u + 1) = (this lane o, partner q).  With
      // sg = +1 on the even lane and -1 on the odd one, the even lane's output is o + q and
      // the odd lane's q - o: sg o + q, both directions.
      const float sg = par ? -1.f : 1.f;
#pragma unroll
      for (int b = 0; b < H / G; ++b) {
        if (b + 1 < H / G) {
#pragma unroll
          for (int t = 0; t < G; ++t) vn[t] = v[(2 * ((b + 1) * G + t) + par) * N2];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < G; ++t) {
          const int u = b * G + t;
          const C o = h[u];
          C y;
          y.x = fmaf(sg, o.x, lane_xor1(o.x)) * vb[t];
          y.y = fmaf(sg, o.y, lane_xor1(o.y)) * vb[t];
          C z;
          z.x = fmaf(sg, y.x, lane_xor1(y.x));
          z.y = fmaf(sg, y.y, lane_xor1(y.y));
          h[u] = z;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < G; ++t) vb[t] = vn[t];
      }
      rstages_half<N1, 0, NS1 - 1, false>(h, twx, par);
    }
#pragma unroll
    for (int u = 0; u < H; ++u) {
      const int x0 = RS * u;
      if (x0 < WX)
        row[x0 * N2S] = h[u];
      else if (x0 >= N1 - WX)
        row[(x0 - XOFF) * N2S] = h[u];
    }
  }
  __syncthreads();
  // y columns, inverse: digit-reversed in, natural out (only the y window is gathered)
  for (int w = threadIdx.x; w < npl * nxa; w += NT) {
    const int p = w / nxa;
    const int c = colc[w - p * nxa];
    if (c < 0) continue;
    C *col = P + p * PS + c * N2S;
    C y[N2];
#pragma unroll
    for (int i = 0; i < N2; ++i) y[i] = col[i];
    rstages<N2, 0, NS2, false>(y, twy);
#pragma unroll
    for (int i = 0; i < N2; ++i)
      if (!YCUT || i < WY || i >= N2 - WY) col[i] = y[i];
  }
  __syncthreads();
  for (int w = threadIdx.x; w < npl * ns; w += NT) {
    const int p = w / ns, s = w - p * ns;
    const int c = wcol(wrap(sx[s] - g0x, N1));
    Sout[so + (size_t)p * ns_pad + s] = c >= 0 ? P[p * PS + c * N2S + wrap(sy[s] - g0y, N2)] : czero<C>();
  }
}

template <int N1, int N2>
__global__ void __launch_bounds__(kThreads) k_plane_to_real(Plane pl, Sticks sk, const KPair *kp, int use_kq,
                                                            int nb, const double2 *__restrict__ Sin, int ns_pad,
                                                            double2 *__restrict__ R) {
  extern __shared__ __align__(16) unsigned char lds[];
  PlaneCtx<N1, N2> pc(pl, lds);
  const int z = blockIdx.x;
  const int item = blockIdx.y;
  const int k = item / nb;
  int e, g0x, g0y, g0z;
  basis_of(kp, k, use_kq, e, g0x, g0y, g0z);
  const EntryDev E = sk.ent[e];
  const int np = pc.np();
  double2 *P = pc.P;
  plane_zero(P, np);
  pc.set_active(sk.xa + E.xa_off, E.nxa, g0x);
  const int *sx = sk.sx + E.st_off;
  const int *sy = sk.sy + E.st_off;
  const size_t so = ((size_t)item * pl.n3 + z) * ns_pad;
  for (int s = threadIdx.x; s < E.ns; s += blockDim.x) P[pc.pos(sx[s], sy[s], g0x, g0y)] = Sin[so + s];
  __syncthreads();
  pc.template y_lines<true>();
  pc.template x_lines<true>();
  double2 *out = R + ((size_t)item * pl.n3 + z) * np;
  for (int i = threadIdx.x; i < np; i += blockDim.x) out[i] = P[i];
}

template <int N1, int N2, class C = double2>
__global__ void __launch_bounds__(kThreads) k_plane_mul_fwd(Plane pl, Sticks sk, const KPair *kp, int nb,
                                                            const C *__restrict__ psi, const C *__restrict__ dv,
                                                            C *__restrict__ Sout, int ns_pad) {
  extern __shared__ __align__(16) unsigned char lds[];
  PlaneCtx<N1, N2, C> pc(pl, lds);
  const int z = blockIdx.x;
  const int item = blockIdx.y;
  const int k = item / nb;
  int e, g0x, g0y, g0z;
  basis_of(kp, k, 1, e, g0x, g0y, g0z);
  const EntryDev E = sk.ent[e];
  const int np = pc.np();
  C *P = pc.P;
  const C *ps = psi + ((size_t)item * pl.n3 + z) * np;
  const C *d = dv + ((size_t)kp[k].spin * pl.n3 + z) * np;
  for (int i = threadIdx.x; i < np; i += blockDim.x) P[i] = cmul(ps[i], d[i]);
  pc.set_active(sk.xa + E.xa_off, E.nxa, g0x);
  pc.template x_lines<false>();
  pc.template y_lines<false>();
  const int *sx = sk.sx + E.st_off;
  const int *sy = sk.sy + E.st_off;
  const size_t so = ((size_t)item * pl.n3 + z) * ns_pad;
  for (int s = threadIdx.x; s < E.ns; s += blockDim.x) Sout[so + s] = P[pc.pos(sx[s], sy[s], g0x, g0y)];
}

template <int N1, int N2, class C = double2>
__global__ void __launch_bounds__(kThreads) k_plane_drho(Plane pl, Sticks sk, const KPair *kp, int nb,
                                                         const C *__restrict__ Sdu, int ns_pad,
                                                         const C *__restrict__ psi, double2 *__restrict__ part,
                                                         int nsplit) {
  extern __shared__ __align__(16) unsigned char lds[];
  PlaneCtx<N1, N2, C> pc(pl, lds);
  const int z = blockIdx.x;
  const int k = blockIdx.y;
  const int split = blockIdx.z;  // bands [v0, v1) of this workgroup
  const int per = (nb + nsplit - 1) / nsplit;
  const int v0 = split * per, v1 = min(nb, v0 + per);
  int e, g0x, g0y, g0z;
  basis_of(kp, k, 1, e, g0x, g0y, g0z);
  const EntryDev E = sk.ent[e];
  const int np = pc.np();
  C *P = pc.P;
  const int *sx = sk.sx + E.st_off;
  const int *sy = sk.sy + E.st_off;
  pc.set_active(sk.xa + E.xa_off, E.nxa, g0x);
  constexpr int PER = N1 > 0 ? (N1 * N2 + kThreads - 1) / kThreads : kMaxPerThread;
  double2 acc[PER];
  for (int j = 0; j < PER; ++j) acc[j] = make_double2(0.0, 0.0);
  for (int v = v0; v < v1; ++v) {
    const int item = k * nb + v;
    plane_zero(P, np);
    __syncthreads();
    const size_t so = ((size_t)item * pl.n3 + z) * ns_pad;
    for (int s = threadIdx.x; s < E.ns; s += blockDim.x) P[pc.pos(sx[s], sy[s], g0x, g0y)] = Sdu[so + s];
    __syncthreads();
    pc.template y_lines<true>();
    pc.template x_lines<true>();
    const C *ps = psi + ((size_t)item * pl.n3 + z) * np;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int i = threadIdx.x + j * blockDim.x;
      if (i < np) {  // product in C, accumulation in FP64
        const C pr = cmulc(P[i], ps[i]);
        acc[j].x += (double)pr.x;
        acc[j].y += (double)pr.y;
      }
    }
    __syncthreads();
  }
  double2 *out = part + (((size_t)k * nsplit + split) * pl.n3 + z) * np;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int i = threadIdx.x + j * blockDim.x;
    if (i < np) out[i] = acc[j];
  }
}

__global__ void k_drho_reduce(const KPair *kp, int nk, int nsplit, const double2 *__restrict__ part, long nr,
                              double inv_omega, double occ, int nspin, double2 *__restrict__ drho) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= nr) return;
  double2 acc[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
  for (int k = 0; k < nk; ++k) {
    const double w = 2.0 * occ * kp[k].weight * inv_omega;
    double2 p = make_double2(0.0, 0.0);
    for (int s = 0; s < nsplit; ++s) {
      const double2 t = part[((size_t)k * nsplit + s) * nr + i];
      p.x += t.x;
      p.y += t.y;
    }
    const int sp = kp[k].spin;
    acc[sp].x += w * p.x;
    acc[sp].y += w * p.y;
  }
  drho[i] = acc[0];
  if (nspin == 2) drho[nr + i] = acc[1];
}

// Hartree step 1: permuted real-space plane -> natural plane of G_x, G_y (forward).
template <int N1, int N2>
__global__ void __launch_bounds__(kThreads) k_hxc_planes_fwd(Plane pl, const double2 *__restrict__ drho,
                                                             int nspin, double2 *__restrict__ tmp) {
  extern __shared__ __align__(16) unsigned char lds[];
  PlaneCtx<N1, N2> pc(pl, lds);
  const int z = blockIdx.x;
  const int np = pc.np();
  double2 *P = pc.P;
  const double2 *in = drho + (size_t)z * np;
  const size_t nr = (size_t)np * pl.n3;
  if (nspin == 2) {  // Hartree of the total response density
    for (int i = threadIdx.x; i < np; i += blockDim.x) P[i] = cadd(in[i], in[nr + i]);
  } else {
    for (int i = threadIdx.x; i < np; i += blockDim.x) P[i] = in[i];
  }
  pc.set_all_x();
  pc.template x_lines<false>();
  pc.template y_lines<false>();
  double2 *out = tmp + (size_t)z * np;
  for (int i = threadIdx.x; i < np; i += blockDim.x) out[i] = P[i];
}

__device__ __forceinline__ int freq_of(int j, int n) { return j < (n + 1) / 2 ? j : j - n; }

// Hartree step 2: along z, forward DFT, multiply by 4 pi / |q+G|^2 / N_r, inverse DFT.
__global__ void k_hxc_columns(Plane pl, const double2 *__restrict__ tw3, const double *__restrict__ bvec,
                              double q0, double q1, double q2, double2 *__restrict__ tmp) {
  extern __shared__ double2 sm[];
  const int n3 = pl.n3;
  const int np = pl.n1 * pl.n2;
  const int cols = blockDim.x;
  const int c0 = blockIdx.x * cols;
  const int c = c0 + threadIdx.x;
  double2 *a = sm;               // [n3][cols] 
  double2 *f = sm + n3 * cols;   // [n3][cols]
  if (c < np)
    for (int z = 0; z < n3; ++z) a[z * cols + threadIdx.x] = tmp[(size_t)z * np + c];
  __syncthreads();
  if (c >= np) return;
  const int x = c / pl.n2, y = c - x * pl.n2;
  const double mx = freq_of(x, pl.n1) + q0, my = freq_of(y, pl.n2) + q1;
  const double inv_nr = 1.0 / ((double)np * n3);
  for (int zz = 0; zz < n3; ++zz) {
    double2 acc = make_double2(0.0, 0.0);
    for (int z = 0; z < n3; ++z) acc = cadd(acc, cmulc(a[z * cols + threadIdx.x], tw3[(z * zz) % n3]));
    const double mz = freq_of(zz, n3) + q2;
    const double gx = mx * bvec[0] + my * bvec[3] + mz * bvec[6];
    const double gy = mx * bvec[1] + my * bvec[4] + mz * bvec[7];
    const double gz = mx * bvec[2] + my * bvec[5] + mz * bvec[8];
    const double g2 = gx * gx + gy * gy + gz * gz;
    const double s = g2 > 1e-12 ? 4.0 * M_PI / g2 * inv_nr : 0.0;
    f[zz * cols + threadIdx.x] = cscale(acc, s);
  }
  for (int z = 0; z < n3; ++z) {
    double2 acc = make_double2(0.0, 0.0);
    for (int zz = 0; zz < n3; ++zz) acc = cadd(acc, cmul(f[zz * cols + threadIdx.x], tw3[(z * zz) % n3]));
    tmp[(size_t)z * np + c] = acc;
  }
}

// Hartree step 3: natural plane -> permuted real space, plus f_xc * drho.
template <int N1, int N2>
__global__ void __launch_bounds__(kThreads) k_hxc_planes_inv(Plane pl, const double2 *__restrict__ tmp,
                                                             const double *__restrict__ fxc,
                                                             const double2 *__restrict__ drho, int nspin,
                                                             double2 *__restrict__ dvout) {
  extern __shared__ __align__(16) unsigned char lds[];
  PlaneCtx<N1, N2> pc(pl, lds);
  const int z = blockIdx.x;
  const int np = pc.np();
  double2 *P = pc.P;
  const double2 *in = tmp + (size_t)z * np;
  for (int i = threadIdx.x; i < np; i += blockDim.x) P[i] = in[i];
  pc.set_all_x();
  pc.template y_lines<true>();
  pc.template x_lines<true>();
  const size_t o = (size_t)z * np;
  if (nspin == 2) {  // dv_s = V_H + f_s,up drho_up + f_s,dn drho_dn; fxc = [f_uu, f_ud, f_dd]
    const size_t nr = (size_t)np * pl.n3;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
      const double fuu = fxc[o + i], fud = fxc[nr + o + i], fdd = fxc[2 * nr + o + i];
      const double2 du = drho[o + i], dd = drho[nr + o + i];
      dvout[o + i] = make_double2(P[i].x + fuu * du.x + fud * dd.x, P[i].y + fuu * du.y + fud * dd.y);
      dvout[nr + o + i] = make_double2(P[i].x + fud * du.x + fdd * dd.x, P[i].y + fud * du.y + fdd * dd.y);
    }
    return;
  }
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    const double fx = fxc[o + i];
    const double2 d = drho[o + i];
    dvout[o + i] = make_double2(P[i].x + fx * d.x, P[i].y + fx * d.y);
  }
}

__global__ void k_permute_real(Plane pl, const int *__restrict__ px, const int *__restrict__ py,
                               const double *__restrict__ in, double *__restrict__ out) {
  // in: [N1][N2][N3] natural; out: [N3][xp][yp]
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long np = (long)pl.n1 * pl.n2;
  if (i >= np * pl.n3) return;
  const int z = (int)(i / np);
  const int r = (int)(i - z * np);
  const int xp = r / pl.n2, yp = r - xp * pl.n2;
  out[i] = in[((long)px[xp] * pl.n2 + py[yp]) * pl.n3 + z];
}

__global__ void k_permute_complex(Plane pl, const int *__restrict__ px, const int *__restrict__ py,
                                  const double2 *__restrict__ in, double2 *__restrict__ out, int inverse) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long np = (long)pl.n1 * pl.n2;
  if (i >= np * pl.n3) return;
  const int z = (int)(i / np);
  const int r = (int)(i - z * np);
  const int xp = r / pl.n2, yp = r - xp * pl.n2;
  const long nat = ((long)px[xp] * pl.n2 + py[yp]) * pl.n3 + z;
  if (inverse)
    out[nat] = in[i];
  else
    out[i] = in[nat];
}

__global__ void k_fxc(const double *__restrict__ rho, double *__restrict__ fxc, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double r = rho[i];
  if (!(r > 1e-10)) {
    fxc[i] = 0.0;
    return;
  }
  // Perdew-Zunger 1981 LDA, spin unpolarized, Hartree units.
  const double gamma = -0.1423, beta1 = 1.0529, beta2 = 0.3334;
  const double A = 0.0311, C = 0.0020, D = -0.0116;
  const double rs = cbrt(3.0 / (4.0 * M_PI * r));
  const double fx = -(1.0 / 3.0) * cbrt(3.0 / M_PI) / cbrt(r * r);
  double dv;
  if (rs >= 1.0) {
    const double sq = sqrt(rs);
    const double num = 1.0 + 7.0 / 6.0 * beta1 * sq + 4.0 / 3.0 * beta2 * rs;
    const double den = 1.0 + beta1 * sq + beta2 * rs;
    const double dnum = 7.0 / 12.0 * beta1 / sq + 4.0 / 3.0 * beta2;
    const double dden = 0.5 * beta1 / sq + beta2;
    dv = gamma * (dnum * den - 2.0 * num * dden) / (den * den * den);
  } else {
    dv = A / rs + 2.0 / 3.0 * C * (log(rs) + 1.0) + (2.0 * D - C) / 3.0;
  }
  fxc[i] = fx + dv * (-rs / (3.0 * r));
}

// One Perdew-Zunger correlation fit (gamma, beta1, beta2 for r_s >= 1; A, B, C, D below):
// eps and its first two r_s derivatives.
struct PzFit {
  double g, b1, b2, a, b, c, d;
};
__device__ void pz_fit(const PzFit &f, double rs, double &e0, double &e1, double &e2) {
  if (rs >= 1.0) {
    const double sq = sqrt(rs);
    const double den = 1.0 + f.b1 * sq + f.b2 * rs;
    const double dd1 = 0.5 * f.b1 / sq + f.b2;
    const double dd2 = -0.25 * f.b1 / (rs * sq);
    e0 = f.g / den;
    e1 = -f.g * dd1 / (den * den);
    e2 = f.g * (2.0 * dd1 * dd1 / (den * den * den) - dd2 / (den * den));
  } else {
    const double l = log(rs);
    e0 = f.a * l + f.b + f.c * rs * l + f.d * rs;
    e1 = f.a / rs + f.c * (l + 1.0) + f.d;
    e2 = -f.a / (rs * rs) + f.c / rs;
  }
}

// Collinear spin-polarized LDA kernel d v_s / d rho_t (Hartree units): exchange from the
// spin-scaling relation (diagonal, -(1/3)(6/pi)^(1/3) rho_s^(-2/3)); Perdew-Zunger
// correlation interpolated between the unpolarized and the fully polarized fit with
// f(zeta) = ((1+zeta)^(4/3) + (1-zeta)^(4/3) - 2) / (2^(4/3) - 2), differentiated through
// (r_s, zeta).  Zero where rho_up + rho_dn <= 1e-10; |zeta| clipped at 1 - 1e-12.
__global__ void k_fxc_spin(const double *__restrict__ rup, const double *__restrict__ rdn,
                           double *__restrict__ fxc, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double r = rup[i] + rdn[i];
  if (!(r > 1e-10)) {
    fxc[i] = fxc[n + i] = fxc[2 * n + i] = 0.0;
    return;
  }
  const double zmax = 1.0 - 1e-12;
  const double z = fmin(zmax, fmax(-zmax, (rup[i] - rdn[i]) / r));
  const double rs = cbrt(3.0 / (4.0 * M_PI * r));
  const PzFit fu{-0.1423, 1.0529, 0.3334, 0.0311, -0.048, 0.0020, -0.0116};
  const PzFit fp{-0.0843, 1.3981, 0.2611, 0.01555, -0.0269, 0.0007, -0.0048};
  double u0, u1, u2, p0, p1, p2;
  pz_fit(fu, rs, u0, u1, u2);
  pz_fit(fp, rs, p0, p1, p2);
  const double den = cbrt(16.0) - 2.0;  // 2^(4/3) - 2
  const double cp = cbrt(1.0 + z), cm = cbrt(1.0 - z);
  const double fz = ((1.0 + z) * cp + (1.0 - z) * cm - 2.0) / den;
  const double fz1 = 4.0 / 3.0 * (cp - cm) / den;
  const double fz2 = 4.0 / 9.0 * (1.0 / (cp * cp) + 1.0 / (cm * cm)) / den;
  const double e_r = u1 + fz * (p1 - u1), e_rr = u2 + fz * (p2 - u2);
  const double e_zz = fz2 * (p0 - u0), e_rz = fz1 * (p1 - u1);
  const double a_r = 2.0 / 3.0 * e_r - rs / 3.0 * e_rr;
  const double c6 = cbrt(6.0 / M_PI);
  double f[2][2];
  for (int a = 0; a < 2; ++a) {
    const double sa = a == 0 ? 1.0 : -1.0;
    const double g_rho = -rs / (3.0 * r) * (a_r + (sa - z) * e_rz);   // d/d rho at fixed zeta
    const double g_zeta = -rs / 3.0 * e_rz + (sa - z) * e_zz;        // d/d zeta at fixed rho
    for (int b = 0; b < 2; ++b) {
      const double sb = b == 0 ? 1.0 : -1.0;
      f[a][b] = g_rho + (sb - z) / r * g_zeta;
    }
    const double rsig = 0.5 * r * (1.0 + sa * z);
    f[a][a] += -c6 / (3.0 * cbrt(rsig * rsig));
  }
  fxc[i] = f[0][0];
  fxc[n + i] = 0.5 * (f[0][1] + f[1][0]);
  fxc[2 * n + i] = f[1][1];
}

}  // namespace

// ---------------------------------------------------------------- launchers

// Grid sizes with compile-time transforms; other sizes take the runtime path.
#define COMMA ,
#define HP_PLANE_DISPATCH_T(KERNEL, CT, GRID, LDS, ST, ...)                                                   \
  do {                                                                                                       \
    const int key_ = pl.n1 * 1000 + pl.n2;                                                                  \
    switch (key_) {                                                                                          \
      case 24024: hipLaunchKernelGGL((KERNEL<24, 24 CT>), GRID, dim3(kThreads), LDS, ST, __VA_ARGS__); break;   \
      case 30024: hipLaunchKernelGGL((KERNEL<30, 24 CT>), GRID, dim3(kThreads), LDS, ST, __VA_ARGS__); break;   \
      case 48024: hipLaunchKernelGGL((KERNEL<48, 24 CT>), GRID, dim3(kThreads), LDS, ST, __VA_ARGS__); break;   \
      case 48048: hipLaunchKernelGGL((KERNEL<48, 48 CT>), GRID, dim3(kThreads), LDS, ST, __VA_ARGS__); break;   \
      case 72045: hipLaunchKernelGGL((KERNEL<72, 45 CT>), GRID, dim3(kThreads), LDS, ST, __VA_ARGS__); break;   \
      case 144045: hipLaunchKernelGGL((KERNEL<144, 45 CT>), GRID, dim3(kThreads), LDS, ST, __VA_ARGS__); break; \
      default: hipLaunchKernelGGL((KERNEL<0, 0 CT>), GRID, dim3(kThreads), LDS, ST, __VA_ARGS__); break;        \
    }                                                                                                        \
  } while (0)
#define HP_PLANE_DISPATCH(KERNEL, GRID, LDS, ST, ...) HP_PLANE_DISPATCH_T(KERNEL, , GRID, LDS, ST, __VA_ARGS__)

#define HP_STICK_DISPATCH(KERNEL, CT, GRID, LDS, ST, N3, ...)                                             \
  do {                                                                                                  \
    switch (N3) {                                                                                       \
      case 24: hipLaunchKernelGGL((KERNEL<24, CT>), GRID, dim3(kThreads), LDS, ST, __VA_ARGS__); break;   \
      case 40: hipLaunchKernelGGL((KERNEL<40, CT>), GRID, dim3(kThreads), LDS, ST, __VA_ARGS__); break;   \
      default: hipLaunchKernelGGL((KERNEL<0, CT>), GRID, dim3(kThreads), LDS, ST, __VA_ARGS__); break;    \
    }                                                                                                   \
  } while (0)

template <class C>
hipError_t stick_inv_t(const Sticks &sk, const KPair *kp, int use_kq, int nb, int nitems, const C *X, int ld, C *S,
                       int ns_pad, int n3, const C *tw3, int max_chunk_pw, int ns_max, const int *active, int variant,
                       hipStream_t st) {
  if (variant == 2 && (n3 == 24 || n3 == 40)) {
    dim3 g((ns_max + kThreads - 1) / kThreads, nitems);
    const size_t lds = (size_t)n3 * sizeof(C) + (size_t)sk.max_pw256 * (sizeof(C) + sizeof(int));
    if (n3 == 24)
      hipLaunchKernelGGL((k_stick_inv_sl<24, C>), g, dim3(kThreads), lds, st, sk, kp, use_kq, nb, X, ld, S, ns_pad,
                         tw3, active);
    else
      hipLaunchKernelGGL((k_stick_inv_sl<40, C>), g, dim3(kThreads), lds, st, sk, kp, use_kq, nb, X, ld, S, ns_pad,
                         tw3, active);
    return hipGetLastError();
  }
  if (variant == 1 && (n3 == 24 || n3 == 40)) {
    dim3 g((ns_max + kThreads - 1) / kThreads, nitems);
    if (n3 == 24)
      hipLaunchKernelGGL((k_stick_inv_s<24, C>), g, dim3(kThreads), 0, st, sk, kp, use_kq, nb, X, ld, S, ns_pad, tw3,
                         active);
    else
      hipLaunchKernelGGL((k_stick_inv_s<40, C>), g, dim3(kThreads), 0, st, sk, kp, use_kq, nb, X, ld, S, ns_pad, tw3,
                         active);
    return hipGetLastError();
  }
  dim3 grid((ns_max + kStickChunk - 1) / kStickChunk, nitems);
  size_t lds = (size_t)n3 * sizeof(C) + (size_t)max_chunk_pw * (sizeof(C) + sizeof(int));
  HP_STICK_DISPATCH(k_stick_inv, C, grid, lds, st, n3, sk, kp, use_kq, nb, X, ld, S, ns_pad, n3, tw3, active);
  return hipGetLastError();
}

template <class C>
hipError_t stick_fwd_t(const Sticks &sk, const KPair *kp, int use_kq, int nb, int nitems, const C *S, int ns_pad,
                       int n3, const C *tw3, double scale, C *Y, int ld, int mode, const double *kin,
                       const double *eps, const C *X, int eps_stride, int max_chunk_pw, int ns_max,
                       const int *active, int variant, hipStream_t st) {
  if (variant == 2 && (n3 == 24 || n3 == 40)) {
    dim3 g((ns_max + kThreads - 1) / kThreads, nitems);
    const size_t lds = (size_t)n3 * sizeof(C) + (size_t)sk.max_pw256 * sizeof(C);
    if (n3 == 24)
      hipLaunchKernelGGL((k_stick_fwd_sl<24, C>), g, dim3(kThreads), lds, st, sk, kp, use_kq, nb, S, ns_pad, tw3,
                         scale, Y, ld, mode, kin, eps, X, eps_stride, active);
    else
      hipLaunchKernelGGL((k_stick_fwd_sl<40, C>), g, dim3(kThreads), lds, st, sk, kp, use_kq, nb, S, ns_pad, tw3,
                         scale, Y, ld, mode, kin, eps, X, eps_stride, active);
    return hipGetLastError();
  }
  if (variant == 1 && (n3 == 24 || n3 == 40)) {
    dim3 g((ns_max + kThreads - 1) / kThreads, nitems);
    if (n3 == 24)
      hipLaunchKernelGGL((k_stick_fwd_s<24, C>), g, dim3(kThreads), 0, st, sk, kp, use_kq, nb, S, ns_pad, tw3, scale,
                         Y, ld, mode, kin, eps, X, eps_stride, active);
    else
      hipLaunchKernelGGL((k_stick_fwd_s<40, C>), g, dim3(kThreads), 0, st, sk, kp, use_kq, nb, S, ns_pad, tw3, scale,
                         Y, ld, mode, kin, eps, X, eps_stride, active);
    return hipGetLastError();
  }
  dim3 grid((ns_max + kStickChunk - 1) / kStickChunk, nitems);
  size_t lds = (size_t)n3 * sizeof(C) + (size_t)n3 * kStickChunk * sizeof(C) + (size_t)max_chunk_pw * sizeof(int);
  HP_STICK_DISPATCH(k_stick_fwd, C, grid, lds, st, n3, sk, kp, use_kq, nb, S, ns_pad, n3, tw3, scale, Y, ld, mode,
                    kin, eps, X, eps_stride, active);
  return hipGetLastError();
}

hipError_t launch_stick_inv(const Sticks &sk, const KPair *kp, int use_kq, int nb, int nitems, const double2 *X,
                            int ld, double2 *S, int ns_pad, int n3, const double2 *tw3, int max_chunk_pw, int ns_max,
                            const int *active, int variant, hipStream_t st) {
  return stick_inv_t(sk, kp, use_kq, nb, nitems, X, ld, S, ns_pad, n3, tw3, max_chunk_pw, ns_max, active, variant,
                     st);
}
hipError_t launch_stick_inv32(const Sticks &sk, const KPair *kp, int use_kq, int nb, int nitems, const float2 *X,
                              int ld, float2 *S, int ns_pad, int n3, const float2 *tw3, int max_chunk_pw, int ns_max,
                              const int *active, int variant, hipStream_t st) {
  return stick_inv_t(sk, kp, use_kq, nb, nitems, X, ld, S, ns_pad, n3, tw3, max_chunk_pw, ns_max, active, variant,
                     st);
}

hipError_t launch_stick_fwd(const Sticks &sk, const KPair *kp, int use_kq, int nb, int nitems, const double2 *S,
                            int ns_pad, int n3, const double2 *tw3, double scale, double2 *Y, int ld, int mode,
                            const double *kin, const double *eps, const double2 *X, int eps_stride,
                            int max_chunk_pw, int ns_max, const int *active, int variant, hipStream_t st) {
  return stick_fwd_t(sk, kp, use_kq, nb, nitems, S, ns_pad, n3, tw3, scale, Y, ld, mode, kin, eps, X, eps_stride,
                     max_chunk_pw, ns_max, active, variant, st);
}
hipError_t launch_stick_fwd32(const Sticks &sk, const KPair *kp, int use_kq, int nb, int nitems, const float2 *S,
                              int ns_pad, int n3, const float2 *tw3, double scale, float2 *Y, int ld, int mode,
                              const double *kin, const double *eps, const float2 *X, int eps_stride,
                              int max_chunk_pw, int ns_max, const int *active, int variant, hipStream_t st) {
  return stick_fwd_t(sk, kp, use_kq, nb, nitems, S, ns_pad, n3, tw3, scale, Y, ld, mode, kin, eps, X, eps_stride,
                     max_chunk_pw, ns_max, active, variant, st);
}

constexpr int kLdsBytes = 160 * 1024;  // LDS per CU on gfx950

// Register-resident variants: threads per workgroup, and the LDS header before the planes.
constexpr int kRegThreads[3] = {128, 192, 256};
int reg_lds_header(int n1) { return reg_lds_header_c(n1); }
size_t reg_plane_bytes(const Plane &pl) { return (size_t)reg_cols(pl.n1) * (pl.n2 | 1) * sizeof(float2); }
// Every entry's sphere, shifted by the current pairs' g0, inside the window on x and y.
bool reg_window_ok(const Plane &pl) {
  const int w[2] = {reg_win(pl.n1), reg_win(pl.n2)}, n[2] = {pl.n1, pl.n2};
  for (int a = 0; a < 2; ++a)
    if (2 * w[a] < n[a] && pl.mext[a] + pl.g0ext[a] > w[a]) return false;
  return true;
}
int reg_row_lanes(const Plane &pl) {
  int n = pl.n1, ns = 0, last = 1;
  for (; n > 1; ++ns) {
    last = n % 8 == 0 ? 8 : n % 9 == 0 ? 9 : n % 4 == 0 ? 4 : n % 2 == 0 ? 2 : n % 3 == 0 ? 3 : 5;
    n /= last;
  }
  return (pl.n1 > 72 && last == 2) ? 2 : 1;
}
// z planes per workgroup of a register-resident variant: as many as the y columns and the
// x-row lanes fill the threads, within the LDS.
int reg_planes(const Plane &pl, int variant) {
  const int nt = kRegThreads[variant - 4];
  const int lines = std::max(std::max(pl.nxa_max, 1), pl.n2 * reg_row_lanes(pl));
  int pb = std::max(1, std::min(nt / lines, pl.n3));
  const size_t per = reg_plane_bytes(pl);
  while (pb > 1 && reg_lds_header(pl.n1) + pb * per > (size_t)kLdsBytes) --pb;
  return pb;
}

bool plane_vloc_variant_ok(const Plane &pl, int csize, int variant) {
  const int key = pl.n1 * 1000 + pl.n2;
  const bool shape = key == 72045 || key == 144045 || key == 30024;
  if (variant == 0) return true;
  if (variant == 1 || variant == 2) return shape && pl.n3 % 2 == 0 && plane_lds_t(pl, csize, 2) <= kLdsBytes;
  if (variant == 3) return shape;
  if (variant >= 4 && variant <= 6) {
    const bool ct = key == 24024 || key == 30024 || key == 48024 || key == 48048 || key == 72045 || key == 144045;
    const size_t lds = reg_lds_header(pl.n1) + (size_t)reg_planes(pl, variant) * reg_plane_bytes(pl);
    return csize == (int)sizeof(float2) && ct && pl.nxa_max >= 1 && lds <= (size_t)kLdsBytes && reg_window_ok(pl);
  }
  return false;
}

// Variants of the local-potential round trip: 0 = one plane per 256 threads,
// 1 = two planes per 256 threads, 2 = two planes per 512 threads, 3 = one plane per 256
// threads with the twiddles read from global memory.
namespace {
template <int N1, int N2, class C>
hipError_t plane_vloc_batched(int variant, const Plane &pl, const Sticks &sk, const KPair *kp, int use_kq, int nb,
                              int nitems, const C *Sin, C *Sout, int ns_pad, const RealOf<C> *vp, const int *active,
                              hipStream_t st) {
  if (variant == 3) {
    hipLaunchKernelGGL((k_plane_vloc_b<N1, N2, C, 1, 256, true>), dim3(pl.n3, nitems), dim3(256),
                       plane_lds_t(pl, sizeof(C), 1, true), st, pl, sk, kp, use_kq, nb, Sin, Sout, ns_pad, vp,
                       active);
    return hipGetLastError();
  }
  const size_t lds = plane_lds_t(pl, sizeof(C), 2);
  if (variant == 1)
    hipLaunchKernelGGL((k_plane_vloc_b<N1, N2, C, 2, 256>), dim3(pl.n3 / 2, nitems), dim3(256), lds, st, pl, sk, kp,
                       use_kq, nb, Sin, Sout, ns_pad, vp, active);
  else
    hipLaunchKernelGGL((k_plane_vloc_b<N1, N2, C, 2, 512>), dim3(pl.n3 / 2, nitems), dim3(512), lds, st, pl, sk, kp,
                       use_kq, nb, Sin, Sout, ns_pad, vp, active);
  return hipGetLastError();
}

template <int N1, int N2>
hipError_t plane_vloc_reg(int variant, const Plane &pl, const Sticks &sk, const KPair *kp, int use_kq, int nb,
                          int nitems, const float2 *Sin, float2 *Sout, int ns_pad, const float *vp, const int *active,
                          hipStream_t st) {
  const int pb = reg_planes(pl, variant);
  const size_t lds = reg_lds_header(N1) + (size_t)pb * reg_plane_bytes(pl);
  const dim3 grid((pl.n3 + pb - 1) / pb, nitems);
  switch (kRegThreads[variant - 4]) {
    case 128:
      hipLaunchKernelGGL((k_plane_vloc_r<N1, N2, 128>), grid, dim3(128), lds, st, pl, sk, kp, use_kq, nb, pb, Sin,
                         Sout, ns_pad, vp, active);
      break;
    case 192:
      hipLaunchKernelGGL((k_plane_vloc_r<N1, N2, 192>), grid, dim3(192), lds, st, pl, sk, kp, use_kq, nb, pb, Sin,
                         Sout, ns_pad, vp, active);
      break;
    default:
      hipLaunchKernelGGL((k_plane_vloc_r<N1, N2, 256>), grid, dim3(256), lds, st, pl, sk, kp, use_kq, nb, pb, Sin,
                         Sout, ns_pad, vp, active);
      break;
  }
  return hipGetLastError();
}

template <class C>
hipError_t plane_vloc_t(int variant, const Plane &pl, const Sticks &sk, const KPair *kp, int use_kq, int nb,
                        int nitems, const C *Sin, C *Sout, int ns_pad, const RealOf<C> *vp, const int *active,
                        hipStream_t st) {
  if constexpr (std::is_same<C, float2>::value) {
    if (variant >= 4 && plane_vloc_variant_ok(pl, sizeof(C), variant)) {
      switch (pl.n1 * 1000 + pl.n2) {
        case 24024: return plane_vloc_reg<24, 24>(variant, pl, sk, kp, use_kq, nb, nitems, Sin, Sout, ns_pad, vp, active, st);
        case 30024: return plane_vloc_reg<30, 24>(variant, pl, sk, kp, use_kq, nb, nitems, Sin, Sout, ns_pad, vp, active, st);
        case 48024: return plane_vloc_reg<48, 24>(variant, pl, sk, kp, use_kq, nb, nitems, Sin, Sout, ns_pad, vp, active, st);
        case 48048: return plane_vloc_reg<48, 48>(variant, pl, sk, kp, use_kq, nb, nitems, Sin, Sout, ns_pad, vp, active, st);
        case 72045: return plane_vloc_reg<72, 45>(variant, pl, sk, kp, use_kq, nb, nitems, Sin, Sout, ns_pad, vp, active, st);
        case 144045: return plane_vloc_reg<144, 45>(variant, pl, sk, kp, use_kq, nb, nitems, Sin, Sout, ns_pad, vp, active, st);
        default: break;
      }
    }
  }
  if (variant > 0 && variant < 4 && plane_vloc_variant_ok(pl, sizeof(C), variant)) {
    switch (pl.n1 * 1000 + pl.n2) {
      case 72045:
        return plane_vloc_batched<72, 45, C>(variant, pl, sk, kp, use_kq, nb, nitems, Sin, Sout, ns_pad, vp, active,
                                             st);
      case 144045:
        return plane_vloc_batched<144, 45, C>(variant, pl, sk, kp, use_kq, nb, nitems, Sin, Sout, ns_pad, vp,
                                              active, st);
      case 30024:
        return plane_vloc_batched<30, 24, C>(variant, pl, sk, kp, use_kq, nb, nitems, Sin, Sout, ns_pad, vp, active,
                                             st);
      default:
        break;
    }
  }
  HP_PLANE_DISPATCH_T(k_plane_vloc, COMMA C, dim3(pl.n3, nitems), plane_lds_t(pl, sizeof(C)), st, pl, sk, kp, use_kq,
                      nb, Sin, Sout, ns_pad, vp, active);
  return hipGetLastError();
}
}  // namespace


hipError_t launch_plane_vloc(const Plane &pl, const Sticks &sk, const KPair *kp, int use_kq, int nb, int nitems,
                             const double2 *Sin, double2 *Sout, int ns_pad, const double *vp, const int *active,
                             int variant, hipStream_t st) {
  return plane_vloc_t<double2>(variant, pl, sk, kp, use_kq, nb, nitems, Sin, Sout, ns_pad, vp, active, st);
}
hipError_t launch_plane_vloc32(const Plane &pl, const Sticks &sk, const KPair *kp, int use_kq, int nb, int nitems,
                               const float2 *Sin, float2 *Sout, int ns_pad, const float *vp, const int *active,
                               int variant, hipStream_t st) {
  return plane_vloc_t<float2>(variant, pl, sk, kp, use_kq, nb, nitems, Sin, Sout, ns_pad, vp, active, st);
}

hipError_t launch_plane_to_real(const Plane &pl, const Sticks &sk, const KPair *kp, int use_kq, int nb, int nitems,
                                const double2 *Sin, int ns_pad, double2 *R, hipStream_t st) {
  HP_PLANE_DISPATCH(k_plane_to_real, dim3(pl.n3, nitems), plane_lds_t(pl), st, pl, sk, kp, use_kq, nb, Sin, ns_pad,
                    R);
  return hipGetLastError();
}

hipError_t launch_plane_mul_fwd(const Plane &pl, const Sticks &sk, const KPair *kp, int nb, int nitems,
                                const double2 *psi, const double2 *dv, double2 *Sout, int ns_pad, hipStream_t st) {
  HP_PLANE_DISPATCH(k_plane_mul_fwd, dim3(pl.n3, nitems), plane_lds_t(pl), st, pl, sk, kp, nb, psi, dv, Sout,
                    ns_pad);
  return hipGetLastError();
}
hipError_t launch_plane_mul_fwd32(const Plane &pl, const Sticks &sk, const KPair *kp, int nb, int nitems,
                                  const float2 *psi, const float2 *dv, float2 *Sout, int ns_pad, hipStream_t st) {
  HP_PLANE_DISPATCH_T(k_plane_mul_fwd, COMMA float2, dim3(pl.n3, nitems), plane_lds_t(pl, sizeof(float2)), st, pl,
                      sk, kp, nb, psi, dv, Sout, ns_pad);
  return hipGetLastError();
}

hipError_t launch_plane_drho(const Plane &pl, const Sticks &sk, const KPair *kp, int nb, int nk, const double2 *Sdu,
                             int ns_pad, const double2 *psi, double2 *part, int nsplit, hipStream_t st) {
  if (pl.n1 * pl.n2 > kMaxPerThread * kThreads || nsplit < 1) return hipErrorInvalidValue;
  HP_PLANE_DISPATCH(k_plane_drho, dim3(pl.n3, nk, nsplit), plane_lds_t(pl), st, pl, sk, kp, nb, Sdu, ns_pad, psi,
                    part, nsplit);
  return hipGetLastError();
}
hipError_t launch_plane_drho32(const Plane &pl, const Sticks &sk, const KPair *kp, int nb, int nk, const float2 *Sdu,
                               int ns_pad, const float2 *psi, double2 *part, int nsplit, hipStream_t st) {
  if (pl.n1 * pl.n2 > kMaxPerThread * kThreads || nsplit < 1) return hipErrorInvalidValue;
  HP_PLANE_DISPATCH_T(k_plane_drho, COMMA float2, dim3(pl.n3, nk, nsplit), plane_lds_t(pl, sizeof(float2)), st, pl,
                      sk, kp, nb, Sdu, ns_pad, psi, part, nsplit);
  return hipGetLastError();
}

hipError_t launch_drho_reduce(const KPair *kp, int nk, int nsplit, const double2 *part, long nr, double inv_omega,
                              double occ, int nspin, double2 *drho, hipStream_t st) {
  hipLaunchKernelGGL(k_drho_reduce, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, kp, nk, nsplit, part, nr,
                     inv_omega, occ, nspin, drho);
  return hipGetLastError();
}

hipError_t launch_hxc(const Plane &pl, const Axis &az, const double *bvec, const double *q, const double2 *drho,
                      const double *fxc, double2 *tmp, double2 *dvout, int nspin, hipStream_t st) {
  HP_PLANE_DISPATCH(k_hxc_planes_fwd, dim3(pl.n3), plane_lds_t(pl), st, pl, drho, nspin, tmp);
  const int cols = 32;
  const int np = pl.n1 * pl.n2;
  hipLaunchKernelGGL(k_hxc_columns, dim3((np + cols - 1) / cols), dim3(cols), 2 * pl.n3 * cols * sizeof(double2), st,
                     pl, az.tw, bvec, q[0], q[1], q[2], tmp);
  HP_PLANE_DISPATCH(k_hxc_planes_inv, dim3(pl.n3), plane_lds_t(pl), st, pl, tmp, fxc, drho, nspin, dvout);
  return hipGetLastError();
}

hipError_t launch_permute_real(const Plane &pl, const int *px, const int *py, const double *in, double *out,
                               hipStream_t st) {
  long n = (long)pl.n1 * pl.n2 * pl.n3;
  hipLaunchKernelGGL(k_permute_real, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pl, px, py, in, out);
  return hipGetLastError();
}

hipError_t launch_permute_complex(const Plane &pl, const int *px, const int *py, const double2 *in, double2 *out,
                                  int inverse, hipStream_t st) {
  long n = (long)pl.n1 * pl.n2 * pl.n3;
  hipLaunchKernelGGL(k_permute_complex, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pl, px, py, in, out,
                     inverse);
  return hipGetLastError();
}

hipError_t launch_fxc(const double *rho, double *fxc, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_fxc, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rho, fxc, n);
  return hipGetLastError();
}

hipError_t launch_fxc_spin(const double *rho_up, const double *rho_dn, double *fxc, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_fxc_spin, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rho_up, rho_dn, fxc, n);
  return hipGetLastError();
}

}  // namespace hp
