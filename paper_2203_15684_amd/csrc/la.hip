// Dense linear algebra of the Sternheimer path on gfx950: complex projection /
// expansion GEMMs on the matrix cores (FP64 v_mfma_f64_16x16x4, FP32
// v_mfma_f32_16x16x4, BF16 v_mfma_f32_16x16x16_bf16 with FP32 accumulation), the
// batched preconditioned CG vector updates with per-band FP64 wavefront reductions,
// the mixed-precision residual and refinement kernels, the response-occupation
// contraction and the mixing reductions.  Every reduction runs in a fixed order, so
// results are bitwise reproducible for a given launch shape.
#include "hp_internal.h"

namespace hp {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Lane layouts (measured on gfx950):
//   v_mfma_f64_16x16x4f64: A lane l -> A[l%16][l/16], B lane l -> B[l/16][l%16],
//                          D lane l, element r -> D[l/16 + 4r][l%16]
//   v_mfma_f32_16x16x4f32: same A and B; D lane l, element r -> D[4(l/16) + r][l%16]
__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <class T>
struct Mf;
template <>
struct Mf<double> {
  using acc = d4;
  using c2 = double2;
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mf<float> {
  using acc = f4;
  using c2 = float2;
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <class C>
__device__ __forceinline__ C zc() {
  C r;
  r.x = 0;
  r.y = 0;
  return r;
}

constexpr int kKb = 16;     // K step staged through LDS
constexpr int kPad = 1;     // LDS row padding (complex elements)

// Workgroups go to the eight XCDs round robin (linear id mod 8), each XCD with its own L2.
// The GEMM grids are one-dimensional: the tiles of a group, which read the same operand
// slabs, take consecutive slots on one XCD, so each slab comes from HBM once into that L2.
__device__ __forceinline__ bool xcd_tile(int n_inner, int n_groups, int &inner, int &group) {
  const int L = blockIdx.x, xcd = L & 7, s = L >> 3;
  inner = s % n_inner;
  group = (s / n_inner) * 8 + xcd;
  return group < n_groups;
}
inline unsigned xcd_grid(int n_inner, int n_groups) { return 8u * (unsigned)n_inner * ((n_groups + 7) / 8); }

// C[k][m][v] (partial over a K split) = sum_G conj(T[m0+m][G]) X[v][G].
// Workgroup tile (32 WM rows) x (32 WN bands), four waves in a 2 x 2 arrangement, each
// holding WM x WN 16x16 MFMA blocks; the next K slab is prefetched into registers while
// the current one is multiplied out of LDS.
template <class T, int WM, int WN>
__global__ void __launch_bounds__(256) k_zproj(const KPair *kp, int use_kq, const typename Mf<T>::c2 *__restrict__ Tb,
                                               long t_stride, int m0, int M,
                                               const typename Mf<T>::c2 *__restrict__ X, int ld, int nb,
                                               const int *__restrict__ npw_of, int nsplit,
                                               typename Mf<T>::c2 *__restrict__ Cpart, int nk, const int *bmap,
                                               int nmt, int nnt) {
  using C2 = typename Mf<T>::c2;
  using A4 = typename Mf<T>::acc;
  constexpr int TM = 32 * WM, TN = 32 * WN;
  __shared__ C2 At[TM][kKb + kPad];
  __shared__ C2 Bt[TN][kKb + kPad];
  int inner, group;  // group: (k, K split); inner: (row tile, band tile)
  if (!xcd_tile(nmt * nnt, nk * nsplit, inner, group)) return;
  const int k = group / nsplit;
  const int split = group - k * nsplit;
  const int mt = (inner % nmt) * TM;
  const int nt = (inner / nmt) * TN;
  // band map (nullable): the active bands of each k packed to the front, so tiles cover only
  // those (column j of the tile computes band bm[j]); tiles past the last one exit
  const int *bm = bmap ? bmap + (size_t)k * (nb + 1) + 1 : nullptr;
  const int ncol = bmap ? bm[-1] : nb;
  if (nt >= ncol) return;
  const KPair P = kp[k];
  const int e = use_kq ? P.ej : P.ek;
  const int npw = npw_of[e];
  const int chunk = ((npw + nsplit - 1) / nsplit + kKb - 1) / kKb * kKb;
  const int g_begin = split * chunk;
  const int g_end = min(npw, g_begin + chunk);
  const C2 *Te = Tb + (size_t)e * t_stride + (size_t)m0 * ld;
  const C2 *Xk = X + (size_t)k * nb * ld;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  A4 cr[WM][WN], ci[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      cr[i][j] = A4{0, 0, 0, 0};
      ci[i][j] = A4{0, 0, 0, 0};
    }
  const int lr = threadIdx.x >> 4;  // 0..15: row within a 16-row group
  const int lc = threadIdx.x & 15;  // 0..15: K column
  C2 ra[2 * WM], rb[2 * WN];
  int vb[2 * WN];  // band of each loaded column (-1: none)
#pragma unroll
  for (int i = 0; i < 2 * WN; ++i) {
    const int col = nt + lr + 16 * i;
    vb[i] = col < ncol ? (bm ? bm[col] : col) : -1;
  }
  auto load = [&](int g0) {
    const int g = g0 + lc;
#pragma unroll
    for (int i = 0; i < 2 * WM; ++i) {
      const int row = mt + lr + 16 * i;
      ra[i] = (row < M && g < g_end) ? Te[(size_t)row * ld + g] : zc<C2>();
    }
#pragma unroll
    for (int i = 0; i < 2 * WN; ++i) rb[i] = (vb[i] >= 0 && g < g_end) ? Xk[(size_t)vb[i] * ld + g] : zc<C2>();
  };
  if (g_begin < g_end) load(g_begin);
  for (int g0 = g_begin; g0 < g_end; g0 += kKb) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2 * WM; ++i) At[lr + 16 * i][lc] = ra[i];
#pragma unroll
    for (int i = 0; i < 2 * WN; ++i) Bt[lr + 16 * i][lc] = rb[i];
    __syncthreads();
    if (g0 + kKb < g_end) load(g0 + kKb);
#pragma unroll
    for (int kk = 0; kk < kKb; kk += 4) {
      C2 a[WM], b[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) a[i] = At[(wm * WM + i) * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < WN; ++j) b[j] = Bt[(wn * WN + j) * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {  // conj(a) * b
          cr[i][j] = mfma(a[i].x, b[j].x, cr[i][j]);
          cr[i][j] = mfma(a[i].y, b[j].y, cr[i][j]);
          ci[i][j] = mfma(a[i].x, b[j].y, ci[i][j]);
          ci[i][j] = mfma(-a[i].y, b[j].x, ci[i][j]);
        }
    }
  }
  C2 *Cp = Cpart + ((size_t)split * nk + k) * (size_t)M * nb;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = mt + (wm * WM + i) * 16 + Mf<T>::row(lane, r);
        const int v = nt + (wn * WN + j) * 16 + (lane & 15);
        if (m < M && v < ncol) {
          C2 o;
          o.x = cr[i][j][r];
          o.y = ci[i][j][r];
          Cp[(size_t)m * nb + (bm ? bm[v] : v)] = o;
        }
      }
}

template <class C2>
__global__ void k_zproj_reduce(int total, int M, int nb, int nsplit, const C2 *__restrict__ Cpart,
                               const double *__restrict__ row_scale, double gscale, C2 *__restrict__ C) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  double ax = 0.0, ay = 0.0;
  for (int s = 0; s < nsplit; ++s) {
    const C2 p = Cpart[(size_t)s * total + i];
    ax += p.x;
    ay += p.y;
  }
  double sc = gscale;
  if (row_scale) sc *= row_scale[(i / nb) % M];
  C2 o;
  o.x = ax * sc;
  o.y = ay * sc;
  C[i] = o;
}

// Y[v][G] += sum_m T[m0+m][G] C[k][m][v]; workgroup tile (32 BV bands) x 64 plane waves,
// four waves in a 2 x 2 arrangement (16 BV bands x 32 plane waves each), the next m slab
// prefetched into registers.
template <class T, int BV>
__global__ void __launch_bounds__(256) k_zexpand(const KPair *kp, int use_kq, const typename Mf<T>::c2 *__restrict__ Tb,
                                                 long t_stride, int m0, int M,
                                                 const typename Mf<T>::c2 *__restrict__ C, long c_kstride,
                                                 double cscale, typename Mf<T>::c2 *__restrict__ Y, int ld, int nb,
                                                 const int *__restrict__ npw_of, const int *bmap, int nk, int ngt,
                                                 int nvt) {
  using C2 = typename Mf<T>::c2;
  using A4 = typename Mf<T>::acc;
  constexpr int TV = 32 * BV;
  __shared__ C2 Ct[TV][kKb + kPad];  // [v][m]
  __shared__ C2 Tt[kKb][64 + kPad];  // [m][G]
  int inner, group;  // group: (k, plane-wave tile); inner: band tile
  if (!xcd_tile(nvt, nk * ngt, inner, group)) return;
  const int k = group / ngt;
  const int vt = inner * TV;
  const int *bm = bmap ? bmap + (size_t)k * (nb + 1) + 1 : nullptr;  // packed active bands
  const int ncol = bmap ? bm[-1] : nb;
  if (vt >= ncol) return;
  const KPair P = kp[k];
  const int e = use_kq ? P.ej : P.ek;
  const int npw = npw_of[e];
  const int gt = (group - k * ngt) * 64;
  if (gt >= npw) return;
  const C2 *Te = Tb + (size_t)e * t_stride + (size_t)m0 * ld;
  const C2 *Ck = C + (size_t)k * c_kstride;
  const T cs = (T)cscale;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wv = wave >> 1, wg = wave & 1;
  A4 yr[BV][2], yi[BV][2];
#pragma unroll
  for (int i = 0; i < BV; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      yr[i][j] = A4{0, 0, 0, 0};
      yi[i][j] = A4{0, 0, 0, 0};
    }
  C2 rc[2 * BV], rt[4];
  auto load = [&](int mb) {
#pragma unroll
    for (int c = 0; c < 2 * BV; ++c) {  // C slab: TV bands x 16 m
      const int idx = threadIdx.x + 256 * c;
      const int vv = idx % TV, mm = idx / TV;
      const int m = mb + mm, v = vt + vv;
      C2 val = zc<C2>();
      if (m < M && v < ncol) {
        val = Ck[(size_t)m * nb + (bm ? bm[v] : v)];
        val.x *= cs;
        val.y *= cs;
      }
      rc[c] = val;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {  // T slab: 16 m x 64 G
      const int idx = threadIdx.x + c * 256;
      const int mm = idx >> 6, gg = idx & 63;
      const int m = mb + mm, g = gt + gg;
      rt[c] = (m < M && g < npw) ? Te[(size_t)m * ld + g] : zc<C2>();
    }
  };
  load(0);
  for (int mb = 0; mb < M; mb += kKb) {
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 2 * BV; ++c) {
      const int idx = threadIdx.x + 256 * c;
      Ct[idx % TV][idx / TV] = rc[c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int idx = threadIdx.x + c * 256;
      Tt[idx >> 6][idx & 63] = rt[c];
    }
    __syncthreads();
    if (mb + kKb < M) load(mb + kKb);
#pragma unroll
    for (int kk = 0; kk < kKb; kk += 4) {
      const C2 b0 = Tt[kk + (lane >> 4)][wg * 32 + (lane & 15)];
      const C2 b1 = Tt[kk + (lane >> 4)][wg * 32 + 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < BV; ++i) {
        const C2 a = Ct[(wv * BV + i) * 16 + (lane & 15)][kk + (lane >> 4)];
        yr[i][0] = mfma(a.x, b0.x, yr[i][0]);
        yr[i][0] = mfma(-a.y, b0.y, yr[i][0]);
        yi[i][0] = mfma(a.x, b0.y, yi[i][0]);
        yi[i][0] = mfma(a.y, b0.x, yi[i][0]);
        yr[i][1] = mfma(a.x, b1.x, yr[i][1]);
        yr[i][1] = mfma(-a.y, b1.y, yr[i][1]);
        yi[i][1] = mfma(a.x, b1.y, yi[i][1]);
        yi[i][1] = mfma(a.y, b1.x, yi[i][1]);
      }
    }
  }
  C2 *Yk = Y + (size_t)k * nb * ld;
#pragma unroll
  for (int i = 0; i < BV; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int vc = vt + (wv * BV + i) * 16 + Mf<T>::row(lane, r);
      if (vc >= ncol) continue;
      const int v = bm ? bm[vc] : vc;
      const int g = gt + wg * 32 + (lane & 15);
      if (g < npw) {
        C2 y = Yk[(size_t)v * ld + g];
        y.x += yr[i][0][r];
        y.y += yi[i][0][r];
        Yk[(size_t)v * ld + g] = y;
      }
      if (g + 16 < npw) {
        C2 y = Yk[(size_t)v * ld + g + 16];
        y.x += yr[i][1][r];
        y.y += yi[i][1][r];
        Yk[(size_t)v * ld + g + 16] = y;
      }
    }
}

// ---------------------------------------------------------------- BF16 GEMMs
// Projector tables in bfloat16 (one 32-bit word per complex: real part in the low half),
// vectors and accumulation in FP32, on v_mfma_f32_16x16x16_bf16 (measured on gfx950:
// A lane l, value j -> A[l%16][4(l/16)+j]; B lane l, value j -> B[4(l/16)+j][l%16];
// D as for the FP32 instruction).
typedef short s4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_rne(float x) {  // round to nearest even
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ f4 mfma16(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ s4 neg4(s4 a) {
  s4 r;
#pragma unroll
  for (int j = 0; j < 4; ++j) r[j] = (short)(a[j] ^ (short)0x8000);
  return r;
}
constexpr int kKb16 = 32;        // K step per LDS stage (two MFMA k-blocks)
constexpr int kLd16 = kKb16 + 4; // LDS row length in bf16 (8-byte aligned reads of 4 values)

// C[k][m][v] (partial over a K split) = sum_G conj(T16[m0+m][G]) X[v][G], X FP32.
template <int WM, int WN>
__global__ void __launch_bounds__(256) k_zproj16(const KPair *kp, int use_kq, const unsigned *__restrict__ Tb,
                                                 long t_stride, int m0, int M, const float2 *__restrict__ X, int ld,
                                                 int nb, const int *__restrict__ npw_of, int nsplit,
                                                 float2 *__restrict__ Cpart, int nk, const int *bmap, int nmt,
                                                 int nnt) {
  constexpr int TM = 32 * WM, TN = 32 * WN;
  __shared__ __align__(8) short Ar[TM][kLd16], Ai[TM][kLd16], Br[TN][kLd16], Bi[TN][kLd16];
  int inner, group;  // group: (k, K split); inner: (row tile, band tile)
  if (!xcd_tile(nmt * nnt, nk * nsplit, inner, group)) return;
  const int k = group / nsplit;
  const int split = group - k * nsplit;
  const int mt = (inner % nmt) * TM;
  const int nt = (inner / nmt) * TN;
  const int *bm = bmap ? bmap + (size_t)k * (nb + 1) + 1 : nullptr;  // packed active bands
  const int ncol = bmap ? bm[-1] : nb;
  if (nt >= ncol) return;
  const KPair P = kp[k];
  const int e = use_kq ? P.ej : P.ek;
  const int npw = npw_of[e];
  const int chunk = ((npw + nsplit - 1) / nsplit + kKb16 - 1) / kKb16 * kKb16;
  const int g_begin = split * chunk;
  const int g_end = min(npw, g_begin + chunk);
  const unsigned *Te = Tb + (size_t)e * t_stride + (size_t)m0 * ld;
  const float2 *Xk = X + (size_t)k * nb * ld;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  f4 cr[WM][WN], ci[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      cr[i][j] = f4{0, 0, 0, 0};
      ci[i][j] = f4{0, 0, 0, 0};
    }
  const int lr = threadIdx.x >> 5;  // 0..7
  const int lc = threadIdx.x & 31;  // K column
  unsigned ra[4 * WM];
  float2 rb[4 * WN];
  int vb[4 * WN];  // band of each loaded column (-1: none)
#pragma unroll
  for (int i = 0; i < 4 * WN; ++i) {
    const int col = nt + lr + 8 * i;
    vb[i] = col < ncol ? (bm ? bm[col] : col) : -1;
  }
  auto load = [&](int g0) {
    const int g = g0 + lc;
#pragma unroll
    for (int i = 0; i < 4 * WM; ++i) {
      const int row = mt + lr + 8 * i;
      ra[i] = (row < M && g < g_end) ? Te[(size_t)row * ld + g] : 0u;
    }
#pragma unroll
    for (int i = 0; i < 4 * WN; ++i)
      rb[i] = (vb[i] >= 0 && g < g_end) ? Xk[(size_t)vb[i] * ld + g] : make_float2(0.f, 0.f);
  };
  if (g_begin < g_end) load(g_begin);
  for (int g0 = g_begin; g0 < g_end; g0 += kKb16) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4 * WM; ++i) {
      Ar[lr + 8 * i][lc] = (short)(ra[i] & 0xFFFFu);
      Ai[lr + 8 * i][lc] = (short)(ra[i] >> 16);
    }
#pragma unroll
    for (int i = 0; i < 4 * WN; ++i) {
      Br[lr + 8 * i][lc] = (short)bf16_rne(rb[i].x);
      Bi[lr + 8 * i][lc] = (short)bf16_rne(rb[i].y);
    }
    __syncthreads();
    if (g0 + kKb16 < g_end) load(g0 + kKb16);
#pragma unroll
    for (int kk = 0; kk < kKb16; kk += 16) {
      const int kc = kk + 4 * (lane >> 4);
      s4 ar[WM], ai[WM], br[WN], bi[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        const int row = (wm * WM + i) * 16 + (lane & 15);
        ar[i] = *reinterpret_cast<const s4 *>(&Ar[row][kc]);
        ai[i] = *reinterpret_cast<const s4 *>(&Ai[row][kc]);
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int col = (wn * WN + j) * 16 + (lane & 15);
        br[j] = *reinterpret_cast<const s4 *>(&Br[col][kc]);
        bi[j] = *reinterpret_cast<const s4 *>(&Bi[col][kc]);
      }
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        const s4 nai = neg4(ai[i]);
#pragma unroll
        for (int j = 0; j < WN; ++j) {  // conj(a) * b
          cr[i][j] = mfma16(ar[i], br[j], cr[i][j]);
          cr[i][j] = mfma16(ai[i], bi[j], cr[i][j]);
          ci[i][j] = mfma16(ar[i], bi[j], ci[i][j]);
          ci[i][j] = mfma16(nai, br[j], ci[i][j]);
        }
      }
    }
  }
  float2 *Cp = Cpart + ((size_t)split * nk + k) * (size_t)M * nb;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = mt + (wm * WM + i) * 16 + 4 * (lane >> 4) + r;
        const int v = nt + (wn * WN + j) * 16 + (lane & 15);
        if (m < M && v < ncol) Cp[(size_t)m * nb + (bm ? bm[v] : v)] = make_float2(cr[i][j][r], ci[i][j][r]);
      }
}

// Y[v][G] += sum_m T16[m0+m][G] C[k][m][v] (C, Y FP32); tile (32 BV bands) x 64 plane waves.
template <int BV>
__global__ void __launch_bounds__(256) k_zexpand16(const KPair *kp, int use_kq, const unsigned *__restrict__ Tb,
                                                   long t_stride, int m0, int M, const float2 *__restrict__ C,
                                                   long c_kstride, double cscale, float2 *__restrict__ Y, int ld,
                                                   int nb, const int *__restrict__ npw_of, const int *bmap,
                                                   int nk, int ngt, int nvt) {
  constexpr int TV = 32 * BV;
  __shared__ __align__(8) short Cr[TV][kLd16], Ci[TV][kLd16];  // [v][m]
  __shared__ __align__(8) short Tr[64][kLd16], Ti[64][kLd16];  // [G][m]
  int inner, group;  // group: (k, plane-wave tile); inner: band tile
  if (!xcd_tile(nvt, nk * ngt, inner, group)) return;
  const int k = group / ngt;
  const int vt = inner * TV;
  const int *bm = bmap ? bmap + (size_t)k * (nb + 1) + 1 : nullptr;  // packed active bands
  const int ncol = bmap ? bm[-1] : nb;
  if (vt >= ncol) return;
  const KPair P = kp[k];
  const int e = use_kq ? P.ej : P.ek;
  const int npw = npw_of[e];
  const int gt = (group - k * ngt) * 64;
  if (gt >= npw) return;
  const unsigned *Te = Tb + (size_t)e * t_stride + (size_t)m0 * ld;
  const float2 *Ck = C + (size_t)k * c_kstride;
  const float cs = (float)cscale;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wv = wave >> 1, wg = wave & 1;
  f4 yr[BV][2], yi[BV][2];
#pragma unroll
  for (int i = 0; i < BV; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      yr[i][j] = f4{0, 0, 0, 0};
      yi[i][j] = f4{0, 0, 0, 0};
    }
  float2 rc[4 * BV];
  unsigned rt[8];
  auto load = [&](int mb) {
#pragma unroll
    for (int c = 0; c < 4 * BV; ++c) {  // C slab: TV bands x 32 m (consecutive threads: consecutive bands)
      const int idx = threadIdx.x + 256 * c;
      const int vv = idx % TV, mm = idx / TV;
      const int m = mb + mm, v = vt + vv;
      float2 val = make_float2(0.f, 0.f);
      if (m < M && v < ncol) {
        val = Ck[(size_t)m * nb + (bm ? bm[v] : v)];
        val.x *= cs;
        val.y *= cs;
      }
      rc[c] = val;
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {  // T slab: 32 m x 64 G
      const int idx = threadIdx.x + c * 256;
      const int mm = idx >> 6, gg = idx & 63;
      const int m = mb + mm, g = gt + gg;
      rt[c] = (m < M && g < npw) ? Te[(size_t)m * ld + g] : 0u;
    }
  };
  load(0);
  for (int mb = 0; mb < M; mb += kKb16) {
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4 * BV; ++c) {
      const int idx = threadIdx.x + 256 * c;
      Cr[idx % TV][idx / TV] = (short)bf16_rne(rc[c].x);
      Ci[idx % TV][idx / TV] = (short)bf16_rne(rc[c].y);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int idx = threadIdx.x + c * 256;
      Tr[idx & 63][idx >> 6] = (short)(rt[c] & 0xFFFFu);
      Ti[idx & 63][idx >> 6] = (short)(rt[c] >> 16);
    }
    __syncthreads();
    if (mb + kKb16 < M) load(mb + kKb16);
#pragma unroll
    for (int kk = 0; kk < kKb16; kk += 16) {
      const int kc = kk + 4 * (lane >> 4);
      s4 br[2], bi[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int g = wg * 32 + 16 * j + (lane & 15);
        br[j] = *reinterpret_cast<const s4 *>(&Tr[g][kc]);
        bi[j] = *reinterpret_cast<const s4 *>(&Ti[g][kc]);
      }
#pragma unroll
      for (int i = 0; i < BV; ++i) {
        const int v = (wv * BV + i) * 16 + (lane & 15);
        const s4 ar = *reinterpret_cast<const s4 *>(&Cr[v][kc]);
        const s4 ai = *reinterpret_cast<const s4 *>(&Ci[v][kc]);
        const s4 nai = neg4(ai);
#pragma unroll
        for (int j = 0; j < 2; ++j) {  // c * t
          yr[i][j] = mfma16(ar, br[j], yr[i][j]);
          yr[i][j] = mfma16(nai, bi[j], yr[i][j]);
          yi[i][j] = mfma16(ar, bi[j], yi[i][j]);
          yi[i][j] = mfma16(ai, br[j], yi[i][j]);
        }
      }
    }
  }
  float2 *Yk = Y + (size_t)k * nb * ld;
#pragma unroll
  for (int i = 0; i < BV; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int vc = vt + (wv * BV + i) * 16 + 4 * (lane >> 4) + r;
      if (vc >= ncol) continue;
      const int v = bm ? bm[vc] : vc;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int g = gt + wg * 32 + 16 * j + (lane & 15);
        if (g < npw) {
          float2 y = Yk[(size_t)v * ld + g];
          y.x += yr[i][j][r];
          y.y += yi[i][j][r];
          Yk[(size_t)v * ld + g] = y;
        }
      }
    }
}

__global__ void k_to_bf16_pairs(const double2 *__restrict__ in, unsigned *__restrict__ out, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 z = in[i];
  out[i] = (unsigned)bf16_rne((float)z.x) | ((unsigned)bf16_rne((float)z.y) << 16);
}

// ------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the 256 threads of a block, fixed order; every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

template <class C2>
__global__ void __launch_bounds__(256) k_cg_init(const KPair *kp, int nb, const C2 *__restrict__ B,
                                                 C2 *__restrict__ Xv, C2 *__restrict__ R, C2 *__restrict__ P,
                                                 const C2 *__restrict__ AX, int have_x0, const double *__restrict__ diag,
                                                 const double *__restrict__ eps, int ld,
                                                 const int *__restrict__ npw_of, long diag_stride, double *rz,
                                                 double *bn, double *rn, int *active, double tol,
                                                 const int *only, const double *floor_abs) {
  __shared__ double red[8];
  const int item = blockIdx.x;
  if (only && !only[item]) {
    if (threadIdx.x == 0) active[item] = 0;
    return;
  }
  const int k = item / nb;
  const int e = kp[k].ej;
  const int npw = npw_of[e];
  const double ev = eps[item];
  const double *dg = diag + (size_t)e * diag_stride;
  const size_t o = (size_t)item * ld;
  double sb = 0.0, sr = 0.0, srz = 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const C2 b = B[o + g];
    double rx = b.x, ry = b.y;
    if (have_x0) {
      const C2 ax = AX[o + g];
      rx -= ax.x;
      ry -= ax.y;
    } else {
      Xv[o + g] = zc<C2>();
    }
    const double m = 1.0 / (dg[g] - ev);
    C2 r, pz;
    r.x = rx;
    r.y = ry;
    pz.x = m * rx;
    pz.y = m * ry;
    R[o + g] = r;
    P[o + g] = pz;
    sb += (double)b.x * b.x + (double)b.y * b.y;
    sr += rx * rx + ry * ry;
    srz += m * (rx * rx + ry * ry);
  }
  sb = block_sum(sb, red);
  sr = block_sum(sr, red);
  srz = block_sum(srz, red);
  if (threadIdx.x == 0) {
    const double nb_ = sqrt(sb);
    bn[item] = nb_;
    rn[item] = sqrt(sr);
    rz[item] = srz;
    const double thr = floor_abs ? fmax(tol * nb_, floor_abs[item]) : tol * nb_;
    active[item] = (nb_ > 0.0 && sqrt(sr) > thr) ? 1 : 0;
  }
}

template <class C2>
__global__ void __launch_bounds__(256) k_cg_step(const KPair *kp, int nb, C2 *__restrict__ Xv, C2 *__restrict__ R,
                                                 C2 *__restrict__ P, const C2 *__restrict__ AP,
                                                 const double *__restrict__ diag, const double *__restrict__ eps,
                                                 int ld, const int *__restrict__ npw_of, long diag_stride,
                                                 double *rz, const double *bn, double *rn, int *active,
                                                 const double *tol_p, int *n_active, int *n_bad,
                                                 const double *floor_abs) {
  __shared__ double red[8];
  const int item = blockIdx.x;
  if (!active[item]) return;
  const double tol = *tol_p;
  const int k = item / nb;
  const int e = kp[k].ej;
  const int npw = npw_of[e];
  const double ev = eps[item];
  const double *dg = diag + (size_t)e * diag_stride;
  const size_t o = (size_t)item * ld;
  double pap = 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const C2 p = P[o + g], a = AP[o + g];
    pap += (double)p.x * a.x + (double)p.y * a.y;
  }
  pap = block_sum(pap, red);
  const double rz_old = rz[item];
  const double alpha = rz_old / pap;
  double srz = 0.0, srr = 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const C2 p = P[o + g], a = AP[o + g];
    C2 x = Xv[o + g], r = R[o + g];
    x.x += alpha * p.x;
    x.y += alpha * p.y;
    r.x -= alpha * a.x;
    r.y -= alpha * a.y;
    Xv[o + g] = x;
    R[o + g] = r;
    const double m = 1.0 / (dg[g] - ev);
    const double rr = (double)r.x * r.x + (double)r.y * r.y;
    srr += rr;
    srz += m * rr;
  }
  srz = block_sum(srz, red);
  srr = block_sum(srr, red);
  const double beta = srz / rz_old;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const C2 p = P[o + g], r = R[o + g];
    const double m = 1.0 / (dg[g] - ev);
    C2 pn;
    pn.x = m * r.x + beta * p.x;
    pn.y = m * r.y + beta * p.y;
    P[o + g] = pn;
  }
  if (threadIdx.x == 0) {
    rz[item] = srz;
    const double r_ = sqrt(srr);
    rn[item] = r_;
    const double thr = floor_abs ? fmax(tol * bn[item], floor_abs[item]) : tol * bn[item];
    const int still = (r_ > thr && isfinite(r_)) ? 1 : 0;
    active[item] = still;
    if (still) atomicAdd(n_active, 1);
    if (!isfinite(r_)) atomicAdd(n_bad, 1);
  }
}

// Mixed precision: R = B - AX (FP64) with per-item norms and flags; r32 = (float) R.
template <class AXT>
__global__ void __launch_bounds__(256) k_residual64(const KPair *kp, int nb, const double2 *__restrict__ B,
                                                    const AXT *__restrict__ AX, int have_x,
                                                    double2 *__restrict__ R, float2 *__restrict__ R32, int ld,
                                                    const int *__restrict__ npw_of, double *bn, double *rn,
                                                    int *active, double tol, int *count, double *floor_abs) {
  __shared__ double red[8];
  const int item = blockIdx.x;
  const int k = item / nb;
  const int npw = npw_of[kp[k].ej];
  const size_t o = (size_t)item * ld;
  double sb = 0.0, sr = 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const double2 b = B[o + g];
    double2 r = b;
    if (have_x) {
      const AXT a = AX[o + g];
      r.x -= (double)a.x;
      r.y -= (double)a.y;
    }
    R[o + g] = r;
    R32[o + g] = make_float2((float)r.x, (float)r.y);
    sb += b.x * b.x + b.y * b.y;
    sr += r.x * r.x + r.y * r.y;
  }
  sb = block_sum(sb, red);
  sr = block_sum(sr, red);
  if (threadIdx.x == 0) {
    const double b_ = sqrt(sb), r_ = sqrt(sr);
    bn[item] = b_;
    rn[item] = r_;
    if (floor_abs) floor_abs[item] = 0.5 * tol * b_;  // the inner solve need not go below this
    const int a = (b_ > 0.0 && r_ > tol * b_ && isfinite(r_)) ? 1 : 0;
    active[item] = a;
    if (a) atomicAdd(count, 1);
    if (!isfinite(r_)) atomicAdd(count + 1, 1);
  }
}

// X += (double) D32 for the items that were refined (X is zero-initialized when !have_x).
__global__ void k_refine_update(int nb, double2 *__restrict__ X, const float2 *__restrict__ D, int ld,
                                const int *__restrict__ npw_item, const int *refined, int have_x) {
  const int item = blockIdx.y;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ld) return;
  const size_t o = (size_t)item * ld + g;
  double2 x = have_x ? X[o] : make_double2(0.0, 0.0);
  if (refined[item]) {
    const float2 d = D[o];
    x.x += (double)d.x;
    x.y += (double)d.y;
  }
  X[o] = x;
}

// dn[s][m1][m2] = sum_k occ w_k sum_v (B[k][5s+m1][v] conj(A[k][5s+m2][v]) + B[k][5s+m2][v] conj(A[k][5s+m1][v]))
// (summed over the pairs of every spin)
__global__ void k_dn(const KPair *kp, int nk, int nh, int nb, const double2 *__restrict__ A,
                     const double2 *__restrict__ Bm, double occ, double2 *__restrict__ dn) {
  const int M = 5 * nh;
  for (int t = threadIdx.x; t < nh * 25; t += blockDim.x) {
    const int s = t / 25, m1 = (t / 5) % 5, m2 = t % 5;
    double ar = 0.0, ai = 0.0;
    for (int k = 0; k < nk; ++k) {
      const double w = occ * kp[k].weight;
      const double2 *Ak = A + (size_t)kp[k].ek * M * nb;
      const double2 *Bk = Bm + (size_t)k * M * nb;
      double sr = 0.0, si = 0.0;
      for (int v = 0; v < nb; ++v) {
        const double2 b1 = Bk[(size_t)(5 * s + m1) * nb + v], a2 = Ak[(size_t)(5 * s + m2) * nb + v];
        const double2 b2 = Bk[(size_t)(5 * s + m2) * nb + v], a1 = Ak[(size_t)(5 * s + m1) * nb + v];
        sr += b1.x * a2.x + b1.y * a2.y + b2.x * a1.x + b2.y * a1.y;
        si += b1.y * a2.x - b1.x * a2.y + b2.y * a1.x - b2.x * a1.y;
      }
      ar += w * sr;
      ai += w * si;
    }
    dn[t] = make_double2(ar, ai);
  }
}

// partial[blk][i] = sum over this block's range of conj(a_i) b
__global__ void __launch_bounds__(256) k_zdots_partial(int nvec, const double2 *const *a, const double2 *b, long n,
                                                       double2 *partial) {
  __shared__ double red[8];
  const long per = (n + gridDim.x - 1) / gridDim.x;
  const long lo = blockIdx.x * per;
  const long hi = min(n, lo + per);
  for (int i = 0; i < nvec; ++i) {
    const double2 *ai = a[i];
    double sr = 0.0, si = 0.0;
    for (long j = lo + threadIdx.x; j < hi; j += blockDim.x) {
      const double2 x = ai[j], y = b[j];
      sr += x.x * y.x + x.y * y.y;
      si += x.x * y.y - x.y * y.x;
    }
    sr = block_sum(sr, red);
    si = block_sum(si, red);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * nvec + i] = make_double2(sr, si);
  }
}

__global__ void k_zdots_final(int nvec, int nblk, const double2 *partial, double2 *out) {
  const int i = threadIdx.x;
  if (i >= nvec) return;
  double sr = 0.0, si = 0.0;
  for (int b = 0; b < nblk; ++b) {
    sr += partial[(size_t)b * nvec + i].x;
    si += partial[(size_t)b * nvec + i].y;
  }
  out[i] = make_double2(sr, si);
}

__global__ void k_zaxpy_list(long n, double2 *y, int nvec, const double2 *const *x, const double2 *coef) {
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (j >= n) return;
  double2 acc = y[j];
  for (int i = 0; i < nvec; ++i) {
    const double2 c = coef[i], v = x[i][j];
    acc.x += c.x * v.x - c.y * v.y;
    acc.y += c.x * v.y + c.y * v.x;
  }
  y[j] = acc;
}

__global__ void k_zsub(long n, const double2 *a, const double2 *b, double2 *out) {
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (j < n) out[j] = make_double2(a[j].x - b[j].x, a[j].y - b[j].y);
}

__global__ void k_zscale_copy(long n, const double2 *a, double s, double2 *out) {
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (j < n) out[j] = make_double2(s * a[j].x, s * a[j].y);
}

}  // namespace

namespace {
template <class T>
hipError_t zproj_t(const KPair *kp, int use_kq, int nk, const typename Mf<T>::c2 *Tm, long t_stride, int m0, int M,
                   const typename Mf<T>::c2 *X, int ld, int nb, const int *npw_of, typename Mf<T>::c2 *Cpart,
                   int nsplit, const int *bmap, int tile, hipStream_t st) {
  const int wm = (tile & 1) ? 2 : 1, wn = (tile & 2) ? 2 : 1;
  const int nmt = (M + 32 * wm - 1) / (32 * wm), nnt = (nb + 32 * wn - 1) / (32 * wn);
  dim3 grid(xcd_grid(nmt * nnt, nk * nsplit));
  switch (tile) {
    case 1:
      hipLaunchKernelGGL((k_zproj<T, 2, 1>), grid, dim3(256), 0, st, kp, use_kq, Tm, t_stride, m0, M, X, ld, nb,
                         npw_of, nsplit, Cpart, nk, bmap, nmt, nnt);
      break;
    case 2:
      hipLaunchKernelGGL((k_zproj<T, 1, 2>), grid, dim3(256), 0, st, kp, use_kq, Tm, t_stride, m0, M, X, ld, nb,
                         npw_of, nsplit, Cpart, nk, bmap, nmt, nnt);
      break;
    case 3:
      hipLaunchKernelGGL((k_zproj<T, 2, 2>), grid, dim3(256), 0, st, kp, use_kq, Tm, t_stride, m0, M, X, ld, nb,
                         npw_of, nsplit, Cpart, nk, bmap, nmt, nnt);
      break;
    default:
      hipLaunchKernelGGL((k_zproj<T, 1, 1>), grid, dim3(256), 0, st, kp, use_kq, Tm, t_stride, m0, M, X, ld, nb,
                         npw_of, nsplit, Cpart, nk, bmap, nmt, nnt);
      break;
  }
  return hipGetLastError();
}

template <class T>
hipError_t zexpand_t(const KPair *kp, int use_kq, int nk, const typename Mf<T>::c2 *Tm, long t_stride, int m0, int M,
                     const typename Mf<T>::c2 *C, long c_kstride, double cscale, typename Mf<T>::c2 *Y, int ld,
                     int nb, const int *npw_of, int npw_max, const int *bmap, int bv, hipStream_t st) {
  bv = (bv == 2 || bv == 4) ? bv : 1;
  const int ngt = (npw_max + 63) / 64, nvt = (nb + 32 * bv - 1) / (32 * bv);
  dim3 grid(xcd_grid(nvt, nk * ngt));
  switch (bv) {
    case 2:
      hipLaunchKernelGGL((k_zexpand<T, 2>), grid, dim3(256), 0, st, kp, use_kq, Tm, t_stride, m0, M, C, c_kstride,
                         cscale, Y, ld, nb, npw_of, bmap, nk, ngt, nvt);
      break;
    case 4:
      hipLaunchKernelGGL((k_zexpand<T, 4>), grid, dim3(256), 0, st, kp, use_kq, Tm, t_stride, m0, M, C, c_kstride,
                         cscale, Y, ld, nb, npw_of, bmap, nk, ngt, nvt);
      break;
    default:
      hipLaunchKernelGGL((k_zexpand<T, 1>), grid, dim3(256), 0, st, kp, use_kq, Tm, t_stride, m0, M, C, c_kstride,
                         cscale, Y, ld, nb, npw_of, bmap, nk, ngt, nvt);
      break;
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_zproj(const KPair *kp, int use_kq, int nk, const double2 *T, long t_stride, int m0, int M,
                        const double2 *X, int ld, int nb, const int *npw_of, double2 *Cpart, int nsplit,
                        const int *bmap, int tile, hipStream_t st) {
  return zproj_t<double>(kp, use_kq, nk, T, t_stride, m0, M, X, ld, nb, npw_of, Cpart, nsplit, bmap, tile, st);
}
hipError_t launch_zproj32(const KPair *kp, int use_kq, int nk, const float2 *T, long t_stride, int m0, int M,
                          const float2 *X, int ld, int nb, const int *npw_of, float2 *Cpart, int nsplit,
                          const int *bmap, int tile, hipStream_t st) {
  return zproj_t<float>(kp, use_kq, nk, T, t_stride, m0, M, X, ld, nb, npw_of, Cpart, nsplit, bmap, tile, st);
}

hipError_t launch_zproj_reduce(int nk, int M, int nb, int nsplit, const double2 *Cpart, const double *row_scale,
                               double gscale, double2 *C, hipStream_t st) {
  const int total = nk * M * nb;
  hipLaunchKernelGGL(k_zproj_reduce<double2>, dim3((total + 255) / 256), dim3(256), 0, st, total, M, nb, nsplit,
                     Cpart, row_scale, gscale, C);
  return hipGetLastError();
}
hipError_t launch_zproj_reduce32(int nk, int M, int nb, int nsplit, const float2 *Cpart, const double *row_scale,
                                 double gscale, float2 *C, hipStream_t st) {
  const int total = nk * M * nb;
  hipLaunchKernelGGL(k_zproj_reduce<float2>, dim3((total + 255) / 256), dim3(256), 0, st, total, M, nb, nsplit,
                     Cpart, row_scale, gscale, C);
  return hipGetLastError();
}

hipError_t launch_zproj16(const KPair *kp, int use_kq, int nk, const unsigned *T, long t_stride, int m0, int M,
                          const float2 *X, int ld, int nb, const int *npw_of, float2 *Cpart, int nsplit,
                          const int *bmap, int tile, hipStream_t st) {
  const int w = tile == 3 ? 2 : 1;
  const int nmt = (M + 32 * w - 1) / (32 * w), nnt = (nb + 32 * w - 1) / (32 * w);
  dim3 grid(xcd_grid(nmt * nnt, nk * nsplit));
  if (w == 2)
    hipLaunchKernelGGL((k_zproj16<2, 2>), grid, dim3(256), 0, st, kp, use_kq, T, t_stride, m0, M, X, ld, nb, npw_of,
                       nsplit, Cpart, nk, bmap, nmt, nnt);
  else
    hipLaunchKernelGGL((k_zproj16<1, 1>), grid, dim3(256), 0, st, kp, use_kq, T, t_stride, m0, M, X, ld, nb, npw_of,
                       nsplit, Cpart, nk, bmap, nmt, nnt);
  return hipGetLastError();
}

hipError_t launch_zexpand16(const KPair *kp, int use_kq, int nk, const unsigned *T, long t_stride, int m0, int M,
                            const float2 *C, long c_kstride, double cscale, float2 *Y, int ld, int nb,
                            const int *npw_of, int npw_max, const int *bmap, int bv, hipStream_t st) {
  bv = (bv == 2 || bv == 4) ? bv : 1;
  const int ngt = (npw_max + 63) / 64, nvt = (nb + 32 * bv - 1) / (32 * bv);
  dim3 grid(xcd_grid(nvt, nk * ngt));
  switch (bv) {
    case 2:
      hipLaunchKernelGGL((k_zexpand16<2>), grid, dim3(256), 0, st, kp, use_kq, T, t_stride, m0, M, C, c_kstride,
                         cscale, Y, ld, nb, npw_of, bmap, nk, ngt, nvt);
      break;
    case 4:
      hipLaunchKernelGGL((k_zexpand16<4>), grid, dim3(256), 0, st, kp, use_kq, T, t_stride, m0, M, C, c_kstride,
                         cscale, Y, ld, nb, npw_of, bmap, nk, ngt, nvt);
      break;
    default:
      hipLaunchKernelGGL((k_zexpand16<1>), grid, dim3(256), 0, st, kp, use_kq, T, t_stride, m0, M, C, c_kstride,
                         cscale, Y, ld, nb, npw_of, bmap, nk, ngt, nvt);
      break;
  }
  return hipGetLastError();
}

// bmap[k][0] = number of active items of pair k, bmap[k][1 + j] = band of the j-th of them
// (increasing band order); one workgroup per k, ballot prefix counts.
__global__ void __launch_bounds__(256) k_active_map(const int *__restrict__ active, int nb, int *__restrict__ bmap) {
  __shared__ int wsum[4];
  __shared__ int base;
  const int k = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int *out = bmap + (size_t)k * (nb + 1);
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int c0 = 0; c0 < nb; c0 += 256) {
    const int j = c0 + (int)threadIdx.x;
    const int f = j < nb ? active[(size_t)k * nb + j] != 0 : 0;
    const unsigned long long b = __ballot(f);
    if (lane == 0) wsum[wave] = __popcll(b);
    __syncthreads();
    int off = base;
    for (int w = 0; w < wave; ++w) off += wsum[w];
    if (f) out[1 + off + __popcll(b & ((1ull << lane) - 1ull))] = j;
    __syncthreads();
    if (threadIdx.x == 0) base += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = base;
}

hipError_t launch_active_map(const int *active, int nk, int nb, int *bmap, hipStream_t st) {
  hipLaunchKernelGGL(k_active_map, dim3(nk), dim3(256), 0, st, active, nb, bmap);
  return hipGetLastError();
}

hipError_t launch_to_bf16_pairs(const double2 *in, unsigned *out, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16_pairs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

hipError_t launch_zexpand(const KPair *kp, int use_kq, int nk, const double2 *T, long t_stride, int m0, int M,
                          const double2 *C, long c_kstride, double cscale, double2 *Y, int ld, int nb,
                          const int *npw_of, int npw_max, const int *bmap, int bv, hipStream_t st) {
  return zexpand_t<double>(kp, use_kq, nk, T, t_stride, m0, M, C, c_kstride, cscale, Y, ld, nb, npw_of, npw_max,
                           bmap, bv, st);
}
hipError_t launch_zexpand32(const KPair *kp, int use_kq, int nk, const float2 *T, long t_stride, int m0, int M,
                            const float2 *C, long c_kstride, double cscale, float2 *Y, int ld, int nb,
                            const int *npw_of, int npw_max, const int *bmap, int bv, hipStream_t st) {
  return zexpand_t<float>(kp, use_kq, nk, T, t_stride, m0, M, C, c_kstride, cscale, Y, ld, nb, npw_of, npw_max,
                          bmap, bv, st);
}

hipError_t launch_cg_init(const KPair *kp, int nb, int nitems, const double2 *B, double2 *Xv, double2 *R,
                          double2 *P, const double2 *AX, int have_x0, const double *diag, const double *eps, int ld,
                          const int *npw_of, long diag_stride, double *rz, double *bn, double *rn, int *active,
                          double tol, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_init<double2>, dim3(nitems), dim3(256), 0, st, kp, nb, B, Xv, R, P, AX, have_x0, diag, eps,
                     ld, npw_of, diag_stride, rz, bn, rn, active, tol, (const int *)nullptr, (const double *)nullptr);
  return hipGetLastError();
}
hipError_t launch_cg_init32(const KPair *kp, int nb, int nitems, const float2 *B, float2 *Xv, float2 *R, float2 *P,
                            const double *diag, const double *eps, int ld, const int *npw_of, long diag_stride,
                            double *rz, double *bn, double *rn, int *active, double tol, const int *only,
                            const double *floor_abs, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_init<float2>, dim3(nitems), dim3(256), 0, st, kp, nb, B, Xv, R, P, (const float2 *)nullptr,
                     0, diag, eps, ld, npw_of, diag_stride, rz, bn, rn, active, tol, only, floor_abs);
  return hipGetLastError();
}

hipError_t launch_cg_step(const KPair *kp, int nb, int nitems, double2 *Xv, double2 *R, double2 *P,
                          const double2 *AP, const double *diag, const double *eps, int ld, const int *npw_of,
                          long diag_stride, double *rz, const double *bn, double *rn, int *active, const double *tol,
                          int *n_active, int *n_bad, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_step<double2>, dim3(nitems), dim3(256), 0, st, kp, nb, Xv, R, P, AP, diag, eps, ld, npw_of,
                     diag_stride, rz, bn, rn, active, tol, n_active, n_bad, (const double *)nullptr);
  return hipGetLastError();
}
hipError_t launch_cg_step32(const KPair *kp, int nb, int nitems, float2 *Xv, float2 *R, float2 *P, const float2 *AP,
                            const double *diag, const double *eps, int ld, const int *npw_of, long diag_stride,
                            double *rz, const double *bn, double *rn, int *active, const double *tol, int *n_active,
                            int *n_bad, const double *floor_abs, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_step<float2>, dim3(nitems), dim3(256), 0, st, kp, nb, Xv, R, P, AP, diag, eps, ld, npw_of,
                     diag_stride, rz, bn, rn, active, tol, n_active, n_bad, floor_abs);
  return hipGetLastError();
}

__global__ void k_fill_int(int *p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_double(double *p, int n, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_double(double *p, int n, double v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_double, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

// One thread stores the constant-rate device clock (a vector store: the address depends on
// the thread index).
__global__ void k_clock_stamp(unsigned long long *p) { p[threadIdx.x] = (unsigned long long)wall_clock64(); }

hipError_t launch_clock_stamp(unsigned long long *p, hipStream_t st) {
  hipLaunchKernelGGL(k_clock_stamp, dim3(1), dim3(1), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_fill_int(int *p, int n, int v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

__global__ void k_to_f32(const double *__restrict__ in, float *__restrict__ out, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

__global__ void k_to_f64(const float *__restrict__ in, double *__restrict__ out, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)in[i];
}

hipError_t launch_to_f64(const float *in, double *out, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_to_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double *in, float *out, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

hipError_t launch_residual64(const KPair *kp, int nb, int nitems, const double2 *B, const double2 *AX, int have_x,
                             double2 *R, float2 *R32, int ld, const int *npw_of, double *bn, double *rn, int *active,
                             double tol, int *count, double *floor_abs, hipStream_t st) {
  hipLaunchKernelGGL(k_residual64<double2>, dim3(nitems), dim3(256), 0, st, kp, nb, B, AX, have_x, R, R32, ld, npw_of,
                     bn, rn, active, tol, count, floor_abs);
  return hipGetLastError();
}
hipError_t launch_residual64_ax32(const KPair *kp, int nb, int nitems, const double2 *B, const float2 *AX, double2 *R,
                                  float2 *R32, int ld, const int *npw_of, double *bn, double *rn, int *active,
                                  double tol, int *count, double *floor_abs, hipStream_t st) {
  hipLaunchKernelGGL(k_residual64<float2>, dim3(nitems), dim3(256), 0, st, kp, nb, B, AX, 1, R, R32, ld, npw_of, bn,
                     rn, active, tol, count, floor_abs);
  return hipGetLastError();
}

hipError_t launch_refine_update(int nb, int nitems, double2 *X, const float2 *D, int ld, const int *refined,
                                int have_x, hipStream_t st) {
  hipLaunchKernelGGL(k_refine_update, dim3((ld + 255) / 256, nitems), dim3(256), 0, st, nb, X, D, ld,
                     (const int *)nullptr, refined, have_x);
  return hipGetLastError();
}

hipError_t launch_dn(const KPair *kp, int nk, int nh, int nb, const double2 *A, const double2 *B, double occ,
                     double2 *dn, hipStream_t st) {
  hipLaunchKernelGGL(k_dn, dim3(1), dim3(256), 0, st, kp, nk, nh, nb, A, B, occ, dn);
  return hipGetLastError();
}

hipError_t launch_zdots(int nvec, const double2 *const *a, const double2 *b, long n, double2 *partial, double2 *out,
                        hipStream_t st) {
  const int nblk = 256;
  hipLaunchKernelGGL(k_zdots_partial, dim3(nblk), dim3(256), 0, st, nvec, a, b, n, partial);
  hipLaunchKernelGGL(k_zdots_final, dim3(1), dim3(64), 0, st, nvec, nblk, partial, out);
  return hipGetLastError();
}

hipError_t launch_zaxpy_list(long n, double2 *y, int nvec, const double2 *const *x, const double2 *coef,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_zaxpy_list, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, y, nvec, x, coef);
  return hipGetLastError();
}

hipError_t launch_zsub(long n, const double2 *a, const double2 *b, double2 *out, hipStream_t st) {
  hipLaunchKernelGGL(k_zsub, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, b, out);
  return hipGetLastError();
}

__global__ void k_scale_rows(long n, long per, const double *__restrict__ s, double2 *__restrict__ x) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double f = s[i / per];
  double2 v = x[i];
  v.x *= f;
  v.y *= f;
  x[i] = v;
}

hipError_t launch_scale_rows(long n, long per, const double *s, double2 *x, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, per, s, x);
  return hipGetLastError();
}

hipError_t launch_zscale_copy(long n, const double2 *a, double s, double2 *out, hipStream_t st) {
  hipLaunchKernelGGL(k_zscale_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, s, out);
  return hipGetLastError();
}

}  // namespace hp
