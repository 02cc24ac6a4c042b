// Load-time kernels of the ground-state hand-off: the caller's plane-wave tables
// (host arrays staged to the device, or device arrays taken in place) are gathered
// into the internal z-stick order on the device, the Jacobi diagonal of every
// entry is formed from the final stacked projector table, and the local potential
// and density are checked and averaged with a fixed-order reduction.  The same
// kernels serve host and device inputs, so both give bit-identical contexts.
#include "hp_internal.h"

namespace hp {

namespace {

constexpr int kT = 256;

// dst[r][p] = src[r][order[p]] for p < npw; 0 for npw <= p < ld.
__global__ void __launch_bounds__(kT) k_gather_rows(const double2 *__restrict__ src, int npw,
                                                    const int *__restrict__ order, double2 *__restrict__ dst,
                                                    int ld) {
  const int r = blockIdx.y;
  const int p = blockIdx.x * kT + threadIdx.x;
  if (p >= ld) return;
  dst[(size_t)r * ld + p] = p < npw ? src[(size_t)r * npw + order[p]] : make_double2(0.0, 0.0);
}

// dst[r][order[p]] = src[r][p] for p < npw (src rows of length ld, dst rows of length npw):
// the internal stick order back to the caller's plane-wave order.
__global__ void __launch_bounds__(kT) k_scatter_rows(const double2 *__restrict__ src, int ld, int npw,
                                                     const int *__restrict__ order, double2 *__restrict__ dst) {
  const int r = blockIdx.y;
  const int p = blockIdx.x * kT + threadIdx.x;
  if (p >= npw) return;
  dst[(size_t)r * npw + order[p]] = src[(size_t)r * ld + p];
}

// diag[e][p] = kin[e][p] + vmean[spin(e)] + sum_r scale[r] |T_e[r][p]|^2 (rows in order),
// 1 on the padding p >= npw(e).
__global__ void __launch_bounds__(kT) k_diag(const KPair *__restrict__ self, const EntryDev *__restrict__ ent,
                                             const double2 *__restrict__ T, long t_stride, int nrows,
                                             const double *__restrict__ scale, const double *__restrict__ kin,
                                             const double *__restrict__ vmean, int ld, double *__restrict__ diag) {
  const int e = blockIdx.y;
  const int p = blockIdx.x * kT + threadIdx.x;
  if (p >= ld) return;
  const EntryDev E = ent[e];
  double d = 1.0;
  if (p < E.npw) {
    d = kin[E.pw_off + p] + vmean[self[e].spin];
    const double2 *t = T + (size_t)e * t_stride + p;
    for (int r = 0; r < nrows; ++r) {
      const double2 v = t[(size_t)r * ld];
      d += scale[r] * (v.x * v.x + v.y * v.y);
    }
  }
  diag[(size_t)e * ld + p] = d;
}

// out[2b] = sum of block b (n values), out[2b + 1] = number of non-finite values in it;
// one workgroup per block, fixed summation order.
__global__ void __launch_bounds__(kT) k_block_stats(const double *__restrict__ x, long n, double *__restrict__ out) {
  __shared__ double s[kT];
  __shared__ int bad[kT];
  const double *xb = x + (size_t)blockIdx.x * n;
  double acc = 0.0;
  int nb = 0;
  for (long i = threadIdx.x; i < n; i += kT) {
    const double v = xb[i];
    if (isfinite(v))
      acc += v;
    else
      ++nb;
  }
  s[threadIdx.x] = acc;
  bad[threadIdx.x] = nb;
  __syncthreads();
  for (int h = kT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s[threadIdx.x] += s[threadIdx.x + h];
      bad[threadIdx.x] += bad[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = s[0];
    out[2 * blockIdx.x + 1] = (double)bad[0];
  }
}

}  // namespace

hipError_t launch_gather_rows(const double2 *src, int npw, const int *order, int nrows, double2 *dst, int ld,
                              hipStream_t st) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3((ld + kT - 1) / kT, nrows), dim3(kT), 0, st, src, npw, order, dst, ld);
  return hipGetLastError();
}

hipError_t launch_scatter_rows(const double2 *src, int ld, int npw, const int *order, int nrows, double2 *dst,
                               hipStream_t st) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_rows, dim3((npw + kT - 1) / kT, nrows), dim3(kT), 0, st, src, ld, npw, order, dst);
  return hipGetLastError();
}

hipError_t launch_diag(const KPair *self, const EntryDev *ent, int n_entries, const double2 *T, long t_stride,
                       int nrows, const double *scale, const double *kin, const double *vmean, int ld, double *diag,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_diag, dim3((ld + kT - 1) / kT, n_entries), dim3(kT), 0, st, self, ent, T, t_stride, nrows,
                     scale, kin, vmean, ld, diag);
  return hipGetLastError();
}

hipError_t launch_block_stats(const double *x, int nblocks, long n, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_block_stats, dim3(nblocks), dim3(kT), 0, st, x, n, out);
  return hipGetLastError();
}

}  // namespace hp
