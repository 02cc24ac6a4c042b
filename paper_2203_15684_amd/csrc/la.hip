// Dense linear algebra of the Sternheimer path on gfx950: complex FP64
// projection / expansion GEMMs on the FP64 matrix cores (v_mfma_f64_16x16x4),
// the batched preconditioned CG vector updates with per-band FP64 wavefront
// reductions, the response-occupation contraction and the mixing reductions.
// Every reduction runs in a fixed order, so results are bitwise reproducible.
#include "hp_internal.h"

namespace hp {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// Lane layout of v_mfma_f64_16x16x4f64 (measured on gfx950):
//   A operand: lane l holds A[l % 16][l / 16]   (16 rows x 4 k)
//   B operand: lane l holds B[l / 16][l % 16]   (4 k x 16 cols)
//   D        : lane l, element r holds D[l / 16 + 4 r][l % 16]
__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kTile = 32;   // output tile (rows x cols) of the projection GEMM
constexpr int kKb = 16;     // K step staged through LDS
constexpr int kPad = 1;     // LDS row padding (complex elements)

// C[k][m][v] (partial over a K split) = sum_G conj(T[m0+m][G]) X[v][G].
__global__ void __launch_bounds__(256) k_zproj(const KPair *kp, int use_kq, const double2 *__restrict__ T,
                                               long t_stride, int m0, int M, const double2 *__restrict__ X, int ld,
                                               int nb, const int *__restrict__ npw_of, int nsplit,
                                               double2 *__restrict__ Cpart, int nk, const int *active) {
  __shared__ double2 At[kTile][kKb + kPad];
  __shared__ double2 Bt[kTile][kKb + kPad];
  const int k = blockIdx.z / nsplit;
  const int split = blockIdx.z - k * nsplit;
  if (active) {  // skip tiles whose 32 bands are all converged (their outputs are not used)
    const int v = blockIdx.y * kTile + (threadIdx.x & 31);
    const int a = (threadIdx.x < 32 && v < nb) ? active[k * nb + v] : 0;
    if (!__syncthreads_or(a)) return;
  }
  const KPair P = kp[k];
  const int e = use_kq ? P.ej : P.ek;
  const int npw = npw_of[e];
  const int chunk = ((npw + nsplit - 1) / nsplit + kKb - 1) / kKb * kKb;
  const int g_begin = split * chunk;
  const int g_end = min(npw, g_begin + chunk);
  const int mt = blockIdx.x * kTile;
  const int nt = blockIdx.y * kTile;
  const double2 *Te = T + (size_t)e * t_stride + (size_t)m0 * ld;
  const double2 *Xk = X + (size_t)k * nb * ld;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  d4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
  const int lr = threadIdx.x >> 3;       // 0..31 row for loads
  const int lc = (threadIdx.x & 7) * 2;  // 0..14 column pair
  for (int g0 = g_begin; g0 < g_end; g0 += kKb) {
    for (int c = 0; c < 2; ++c) {
      const int g = g0 + lc + c;
      const int row = mt + lr;
      At[lr][lc + c] = (row < M && g < g_end) ? Te[(size_t)row * ld + g] : make_double2(0.0, 0.0);
      const int col = nt + lr;
      Bt[lr][lc + c] = (col < nb && g < g_end) ? Xk[(size_t)col * ld + g] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kKb; kk += 4) {
      const double2 a = At[wm * 16 + (lane & 15)][kk + (lane >> 4)];
      const double2 b = Bt[wn * 16 + (lane & 15)][kk + (lane >> 4)];
      // conj(a) * b
      cr = mfma(a.x, b.x, cr);
      cr = mfma(a.y, b.y, cr);
      ci = mfma(a.x, b.y, ci);
      ci = mfma(-a.y, b.x, ci);
    }
    __syncthreads();
  }
  double2 *Cp = Cpart + ((size_t)split * nk + k) * (size_t)M * nb;
  for (int r = 0; r < 4; ++r) {
    const int m = mt + wm * 16 + (lane >> 4) + 4 * r;
    const int v = nt + wn * 16 + (lane & 15);
    if (m < M && v < nb) Cp[(size_t)m * nb + v] = make_double2(cr[r], ci[r]);
  }
}

__global__ void k_zproj_reduce(int total, int M, int nb, int nsplit, const double2 *__restrict__ Cpart,
                               const double *__restrict__ row_scale, double gscale, double2 *__restrict__ C) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int s = 0; s < nsplit; ++s) {
    const double2 p = Cpart[(size_t)s * total + i];
    acc.x += p.x;
    acc.y += p.y;
  }
  double sc = gscale;
  if (row_scale) sc *= row_scale[(i / nb) % M];
  C[i] = make_double2(acc.x * sc, acc.y * sc);
}

// Y[v][G] += sum_m T[m0+m][G] C[k][m][v]; tile 32 bands x 64 plane waves.
__global__ void __launch_bounds__(256) k_zexpand(const KPair *kp, int use_kq, const double2 *__restrict__ T,
                                                 long t_stride, int m0, int M, const double2 *__restrict__ C,
                                                 long c_kstride, double cscale, double2 *__restrict__ Y, int ld,
                                                 int nb, const int *__restrict__ npw_of, const int *active) {
  __shared__ double2 Ct[32][kKb + kPad];   // [v][m]
  __shared__ double2 Tt[kKb][64 + kPad];   // [m][G]
  const int k = blockIdx.z;
  if (active) {
    const int v = blockIdx.y * 32 + (threadIdx.x & 31);
    const int a = (threadIdx.x < 32 && v < nb) ? active[k * nb + v] : 0;
    if (!__syncthreads_or(a)) return;
  }
  const KPair P = kp[k];
  const int e = use_kq ? P.ej : P.ek;
  const int npw = npw_of[e];
  const int gt = blockIdx.x * 64;
  if (gt >= npw) return;
  const int vt = blockIdx.y * 32;
  const double2 *Te = T + (size_t)e * t_stride + (size_t)m0 * ld;
  const double2 *Ck = C + (size_t)k * c_kstride;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wv = wave >> 1, wg = wave & 1;
  d4 yr0 = {0, 0, 0, 0}, yi0 = {0, 0, 0, 0}, yr1 = {0, 0, 0, 0}, yi1 = {0, 0, 0, 0};
  for (int mb = 0; mb < M; mb += kKb) {
    // C tile: 32 v x 16 m  (512 values, 2 per thread)
    for (int c = 0; c < 2; ++c) {
      const int idx = threadIdx.x * 2 + c;
      const int vv = idx >> 4, mm = idx & 15;
      const int m = mb + mm, v = vt + vv;
      Ct[vv][mm] = (m < M && v < nb) ? make_double2(cscale * Ck[(size_t)m * nb + v].x, cscale * Ck[(size_t)m * nb + v].y)
                                     : make_double2(0.0, 0.0);
    }
    // T tile: 16 m x 64 G (1024 values, 4 per thread)
    for (int c = 0; c < 4; ++c) {
      const int idx = threadIdx.x + c * 256;
      const int mm = idx >> 6, gg = idx & 63;
      const int m = mb + mm, g = gt + gg;
      Tt[mm][gg] = (m < M && g < npw) ? Te[(size_t)m * ld + g] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kKb; kk += 4) {
      const double2 a = Ct[wv * 16 + (lane & 15)][kk + (lane >> 4)];
      const double2 b0 = Tt[kk + (lane >> 4)][wg * 32 + (lane & 15)];
      const double2 b1 = Tt[kk + (lane >> 4)][wg * 32 + 16 + (lane & 15)];
      yr0 = mfma(a.x, b0.x, yr0);
      yr0 = mfma(-a.y, b0.y, yr0);
      yi0 = mfma(a.x, b0.y, yi0);
      yi0 = mfma(a.y, b0.x, yi0);
      yr1 = mfma(a.x, b1.x, yr1);
      yr1 = mfma(-a.y, b1.y, yr1);
      yi1 = mfma(a.x, b1.y, yi1);
      yi1 = mfma(a.y, b1.x, yi1);
    }
    __syncthreads();
  }
  double2 *Yk = Y + (size_t)k * nb * ld;
  for (int r = 0; r < 4; ++r) {
    const int v = vt + wv * 16 + (lane >> 4) + 4 * r;
    if (v >= nb) continue;
    const int g = gt + wg * 32 + (lane & 15);
    if (g < npw) {
      double2 y = Yk[(size_t)v * ld + g];
      Yk[(size_t)v * ld + g] = make_double2(y.x + yr0[r], y.y + yi0[r]);
    }
    if (g + 16 < npw) {
      double2 y = Yk[(size_t)v * ld + g + 16];
      Yk[(size_t)v * ld + g + 16] = make_double2(y.x + yr1[r], y.y + yi1[r]);
    }
  }
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

__global__ void __launch_bounds__(256) k_cg_init(const KPair *kp, int nb, const double2 *__restrict__ B,
                                                 double2 *__restrict__ Xv, double2 *__restrict__ R,
                                                 double2 *__restrict__ P, const double2 *__restrict__ AX,
                                                 int have_x0, const double *__restrict__ diag,
                                                 const double *__restrict__ eps, int ld,
                                                 const int *__restrict__ npw_of, long diag_stride, double *rz,
                                                 double *bn, double *rn, int *active, double tol) {
  __shared__ double red[8];
  const int item = blockIdx.x;
  const int k = item / nb;
  const int e = kp[k].ej;
  const int npw = npw_of[e];
  const double ev = eps[item];
  const double *dg = diag + (size_t)e * diag_stride;
  const size_t o = (size_t)item * ld;
  double sb = 0.0, sr = 0.0, srz = 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const double2 b = B[o + g];
    double2 r = b;
    if (have_x0) {
      const double2 ax = AX[o + g];
      r = make_double2(b.x - ax.x, b.y - ax.y);
    } else {
      Xv[o + g] = make_double2(0.0, 0.0);
    }
    const double m = 1.0 / (dg[g] - ev);
    R[o + g] = r;
    P[o + g] = make_double2(m * r.x, m * r.y);
    sb += b.x * b.x + b.y * b.y;
    sr += r.x * r.x + r.y * r.y;
    srz += m * (r.x * r.x + r.y * r.y);
  }
  sb = block_sum(sb, red);
  sr = block_sum(sr, red);
  srz = block_sum(srz, red);
  if (threadIdx.x == 0) {
    const double nb_ = sqrt(sb);
    bn[item] = nb_;
    rn[item] = sqrt(sr);
    rz[item] = srz;
    active[item] = (nb_ > 0.0 && sqrt(sr) > tol * nb_) ? 1 : 0;
  }
}

__global__ void __launch_bounds__(256) k_cg_step(const KPair *kp, int nb, double2 *__restrict__ Xv,
                                                 double2 *__restrict__ R, double2 *__restrict__ P,
                                                 const double2 *__restrict__ AP, const double *__restrict__ diag,
                                                 const double *__restrict__ eps, int ld,
                                                 const int *__restrict__ npw_of, long diag_stride, double *rz,
                                                 const double *bn, double *rn, int *active, double tol,
                                                 int *count) {
  __shared__ double red[8];
  const int item = blockIdx.x;
  if (!active[item]) return;
  const int k = item / nb;
  const int e = kp[k].ej;
  const int npw = npw_of[e];
  const double ev = eps[item];
  const double *dg = diag + (size_t)e * diag_stride;
  const size_t o = (size_t)item * ld;
  double pap = 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const double2 p = P[o + g], a = AP[o + g];
    pap += p.x * a.x + p.y * a.y;
  }
  pap = block_sum(pap, red);
  const double rz_old = rz[item];
  const double alpha = rz_old / pap;
  double srz = 0.0, srr = 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const double2 p = P[o + g], a = AP[o + g];
    double2 x = Xv[o + g], r = R[o + g];
    x.x += alpha * p.x;
    x.y += alpha * p.y;
    r.x -= alpha * a.x;
    r.y -= alpha * a.y;
    Xv[o + g] = x;
    R[o + g] = r;
    const double m = 1.0 / (dg[g] - ev);
    const double rr = r.x * r.x + r.y * r.y;
    srr += rr;
    srz += m * rr;
  }
  srz = block_sum(srz, red);
  srr = block_sum(srr, red);
  const double beta = srz / rz_old;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const double2 p = P[o + g], r = R[o + g];
    const double m = 1.0 / (dg[g] - ev);
    P[o + g] = make_double2(m * r.x + beta * p.x, m * r.y + beta * p.y);
  }
  if (threadIdx.x == 0) {
    rz[item] = srz;
    const double r_ = sqrt(srr);
    rn[item] = r_;
    const int still = (r_ > tol * bn[item] && isfinite(r_)) ? 1 : 0;
    active[item] = still;
    if (still) atomicAdd(count, 1);
    if (!isfinite(r_)) atomicAdd(count + 1, 1);
  }
}

// dn[s][m1][m2] = sum_k 2 w_k sum_v (B[k][5s+m1][v] conj(A[k][5s+m2][v]) + B[k][5s+m2][v] conj(A[k][5s+m1][v]))
__global__ void k_dn(const KPair *kp, int nk, int nh, int nb, const double2 *__restrict__ A,
                     const double2 *__restrict__ Bm, double2 *__restrict__ dn) {
  const int M = 5 * nh;
  for (int t = threadIdx.x; t < nh * 25; t += blockDim.x) {
    const int s = t / 25, m1 = (t / 5) % 5, m2 = t % 5;
    double ar = 0.0, ai = 0.0;
    for (int k = 0; k < nk; ++k) {
      const double w = 2.0 * kp[k].weight;
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

hipError_t launch_zproj(const KPair *kp, int use_kq, int nk, const double2 *T, long t_stride, int m0, int M,
                        const double2 *X, int ld, int nb, const int *npw_of, double2 *Cpart, int nsplit,
                        const int *active, hipStream_t st) {
  dim3 grid((M + kTile - 1) / kTile, (nb + kTile - 1) / kTile, nk * nsplit);
  hipLaunchKernelGGL(k_zproj, grid, dim3(256), 0, st, kp, use_kq, T, t_stride, m0, M, X, ld, nb, npw_of, nsplit,
                     Cpart, nk, active);
  return hipGetLastError();
}

hipError_t launch_zproj_reduce(int nk, int M, int nb, int nsplit, const double2 *Cpart, const double *row_scale,
                               double gscale, double2 *C, hipStream_t st) {
  const int total = nk * M * nb;
  hipLaunchKernelGGL(k_zproj_reduce, dim3((total + 255) / 256), dim3(256), 0, st, total, M, nb, nsplit, Cpart,
                     row_scale, gscale, C);
  return hipGetLastError();
}

hipError_t launch_zexpand(const KPair *kp, int use_kq, int nk, const double2 *T, long t_stride, int m0, int M,
                          const double2 *C, long c_kstride, double cscale, double2 *Y, int ld, int nb,
                          const int *npw_of, int npw_max, const int *active, hipStream_t st) {
  dim3 grid((npw_max + 63) / 64, (nb + 31) / 32, nk);
  hipLaunchKernelGGL(k_zexpand, grid, dim3(256), 0, st, kp, use_kq, T, t_stride, m0, M, C, c_kstride, cscale, Y, ld,
                     nb, npw_of, active);
  return hipGetLastError();
}

hipError_t launch_cg_init(const KPair *kp, int nb, int nitems, const double2 *B, double2 *Xv, double2 *R,
                          double2 *P, const double2 *AX, int have_x0, const double *diag, const double *eps, int ld,
                          const int *npw_of, long diag_stride, double *rz, double *bn, double *rn, int *active,
                          double tol, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_init, dim3(nitems), dim3(256), 0, st, kp, nb, B, Xv, R, P, AX, have_x0, diag, eps, ld,
                     npw_of, diag_stride, rz, bn, rn, active, tol);
  return hipGetLastError();
}

hipError_t launch_cg_step(const KPair *kp, int nb, int nitems, double2 *Xv, double2 *R, double2 *P,
                          const double2 *AP, const double *diag, const double *eps, int ld, const int *npw_of,
                          long diag_stride, double *rz, const double *bn, double *rn, int *active, double tol,
                          int *count, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_step, dim3(nitems), dim3(256), 0, st, kp, nb, Xv, R, P, AP, diag, eps, ld, npw_of,
                     diag_stride, rz, bn, rn, active, tol, count);
  return hipGetLastError();
}

hipError_t launch_dn(const KPair *kp, int nk, int nh, int nb, const double2 *A, const double2 *B, double2 *dn,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_dn, dim3(1), dim3(256), 0, st, kp, nk, nh, nb, A, B, dn);
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

hipError_t launch_zscale_copy(long n, const double2 *a, double s, double2 *out, hipStream_t st) {
  hipLaunchKernelGGL(k_zscale_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, s, out);
  return hipGetLastError();
}

}  // namespace hp
