// Internal declarations of the HIP Hubbard-response library: device data
// layout, kernel launchers and the context.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "hp.h"

namespace hp {

// ---------------------------------------------------------------- FFT axes
// In-place mixed-radix FFT along one grid axis: radices in decimation-in-
// frequency order, span[s] = N / (rad[0] * ... * rad[s]).  tw[k] = e^{+2 pi i k/N}.
struct Axis {
  int n;
  int nst;
  int rad[8];
  int span[8];
  const double2 *tw;
  const float2 *tw32;  // the same table rounded to FP32
};

// Plane geometry shared by every plane kernel: the xy plane (N1 x N2, y fastest)
// of one z index.  Real-space arrays live as [N3][N1*N2] with x and y stored in
// the digit-reversed order produced by the decimation-in-frequency transform.
struct Plane {
  Axis ax;   // x = first grid index, length N1, stride N2
  Axis ay;   // y = second grid index, length N2, stride 1
  int n1, n2, n3;
  int nxa_max;  // most active x columns (x holding sticks) of any entry
  int mext[2];  // x and y: largest max(m + 1, -m) of any entry's Miller indices
  int g0ext[2]; // x and y: largest |g0| of the current k+q pairs (0 before any)
};

// Per k-entry geometry (device arrays, flat with offsets).
struct EntryDev {
  int npw;      // plane waves
  int ns;       // z-sticks (distinct (m1, m2) columns)
  int nxa;      // distinct x columns among the sticks
  int pw_off;   // offset into per-plane-wave arrays
  int st_off;   // offset into per-stick arrays
  int xa_off;   // offset into the active-x array
};

// One mesh k of a (site, q) problem: its own entry, the entry holding k+q and the
// reciprocal vector g0 with k + q = k_j + g0 (the k+q basis is entry j shifted by -g0),
// and the spin channel of both (selects the spin's local and response potentials).
struct KPair {
  int ek;
  int ej;
  int g0[3];
  int spin;
  double weight;
};

// Stick tables of all entries (device).
struct Sticks {
  const int *sx;      // [st] grid x of the stick (m1 mod N1, unshifted)
  const int *sy;      // [st] grid y
  const int *sstart;  // [st] first plane wave of the stick (internal order)
  const int *slen;    // [st] plane waves in the stick
  const int *iz;      // [pw] m3 mod N3
  const int *xa;      // [xa] active x columns
  const EntryDev *ent;
  int max_pw256;      // most plane waves in 256 consecutive sticks of any entry
};

// ----------------------------------------------------------------- launchers
// Every launcher enqueues on `st` and returns hipGetLastError().
// Items are (mesh k, band) pairs, item = k * nb + v; the basis of an item is entry
// kp[k].ej shifted by -g0 (use_kq = 1) or entry kp[k].ek (use_kq = 0).

// S[item][z][s] = sum_{G in stick s} X[item][G] e^{+i G_z z}
hipError_t launch_stick_inv(const Sticks &sk, const KPair *kp, int use_kq, int nb, int nitems, const double2 *X,
                            int ld, double2 *S, int ns_pad, int n3, const double2 *tw3, int max_chunk_pw, int ns_max,
                            const int *active, int variant, hipStream_t st);
// Y[item][G] = scale * sum_z S[item][z][s(G)] e^{-i G_z z}   (S may be null: 0)
//   mode 0 adds (kin[G] - eps[k*eps_stride+v]) X[item][G] (eps may be null: 0)
hipError_t launch_stick_fwd(const Sticks &sk, const KPair *kp, int use_kq, int nb, int nitems, const double2 *S,
                            int ns_pad, int n3, const double2 *tw3, double scale, double2 *Y, int ld, int mode,
                            const double *kin, const double *eps, const double2 *X, int eps_stride, int max_chunk_pw,
                            int ns_max, const int *active, int variant, hipStream_t st);
// variant (both z transforms): 0 = a workgroup per 32 sticks, threads over (z, stick);
// 1 = a thread per stick with its N3 values in registers (N3 = 24 or 40; else as 0);
// 2 = as 1 with the plane waves of the workgroup's 256 sticks staged through LDS by
// coalesced loads (inverse) or stores (forward).  All three give the same results.
// FP32 variants of the three operator kernels (mixed-precision inner solves).
hipError_t launch_stick_inv32(const Sticks &sk, const KPair *kp, int use_kq, int nb, int nitems, const float2 *X,
                              int ld, float2 *S, int ns_pad, int n3, const float2 *tw3, int max_chunk_pw, int ns_max,
                              const int *active, int variant, hipStream_t st);
hipError_t launch_stick_fwd32(const Sticks &sk, const KPair *kp, int use_kq, int nb, int nitems, const float2 *S,
                              int ns_pad, int n3, const float2 *tw3, double scale, float2 *Y, int ld, int mode,
                              const double *kin, const double *eps, const float2 *X, int eps_stride,
                              int max_chunk_pw, int ns_max, const int *active, int variant, hipStream_t st);
hipError_t launch_plane_vloc32(const Plane &pl, const Sticks &sk, const KPair *kp, int use_kq, int nb, int nitems,
                               const float2 *Sin, float2 *Sout, int ns_pad, const float *vp, const int *active,
                               int variant, hipStream_t st);
// Plane round trip for the local potential: sticks -> r (DIF) -> * vp -> sticks (reverse).
// variant: 0 = one z plane per 256-thread workgroup, 1 = two planes per 256 threads,
// 2 = two planes per 512 threads (even N3, two planes in LDS), 3 = one plane with the
// twiddles read from global memory (less LDS per workgroup); 1-3 for some plane sizes.
// FP32 only, compile-time plane sizes: 4, 5, 6 = register-resident lines (a thread holds a
// whole y column, then a whole x row or half of it) with LDS only for the transposes, on
// 128, 192 or 256 threads and as many z planes as fill them.
constexpr int kPlaneVariants = 7;
hipError_t launch_plane_vloc(const Plane &pl, const Sticks &sk, const KPair *kp, int use_kq, int nb, int nitems,
                             const double2 *Sin, double2 *Sout, int ns_pad, const double *vp, const int *active,
                             int variant, hipStream_t st);
bool plane_vloc_variant_ok(const Plane &pl, int complex_bytes, int variant);
// Sticks -> real-space plane (permuted layout), R[item][z][plane].
hipError_t launch_plane_to_real(const Plane &pl, const Sticks &sk, const KPair *kp, int use_kq, int nb, int nitems,
                                const double2 *Sin, int ns_pad, double2 *R, hipStream_t st);
// psi[item] (permuted) * dv (permuted) -> sticks of the k+q basis.
hipError_t launch_plane_mul_fwd(const Plane &pl, const Sticks &sk, const KPair *kp, int nb, int nitems,
                                const double2 *psi, const double2 *dv, double2 *Sout, int ns_pad, hipStream_t st);
// part[k][s][z][plane] = sum over the s-th of nsplit band ranges of conj(psi[k*nb+v]) *
// (sticks of du -> r), k+q basis.
hipError_t launch_plane_drho(const Plane &pl, const Sticks &sk, const KPair *kp, int nb, int nk, const double2 *Sdu,
                             int ns_pad, const double2 *psi, double2 *part, int nsplit, hipStream_t st);
// FP32 transforms and products (FP64 accumulation of the density), for the mixed form.
hipError_t launch_plane_mul_fwd32(const Plane &pl, const Sticks &sk, const KPair *kp, int nb, int nitems,
                                  const float2 *psi, const float2 *dv, float2 *Sout, int ns_pad, hipStream_t st);
hipError_t launch_plane_drho32(const Plane &pl, const Sticks &sk, const KPair *kp, int nb, int nk, const float2 *Sdu,
                               int ns_pad, const float2 *psi, double2 *part, int nsplit, hipStream_t st);
// out[i] = (double) in[i]
hipError_t launch_to_f64(const float *in, double *out, long n, hipStream_t st);
// drho = sum_k (4 w_k / Omega) sum_s part[k][s] in fixed order.
// drho[s][i] = (2 occ / Omega) sum over pairs k of spin s of w_k sum_split part[k][split][i]
// (occ electrons per state, 2 for time reversal); s < nspin.
hipError_t launch_drho_reduce(const KPair *kp, int nk, int nsplit, const double2 *part, long nr, double inv_omega,
                              double occ, int nspin, double2 *drho, hipStream_t st);
// dvout = IFFT(4 pi FFT(drho) / |q+G|^2) + fxc * drho, permuted layout.  nspin = 2: drho,
// dvout are [2][nr], the Hartree term uses drho[0] + drho[1] and fxc is [3][nr]
// (f_uu, f_ud, f_dd): dvout[s] = V_H + f_s0 drho[0] + f_s1 drho[1].
hipError_t launch_hxc(const Plane &pl, const Axis &az, const double *bvec, const double *q, const double2 *drho,
                      const double *fxc, double2 *tmp, double2 *dvout, int nspin, hipStream_t st);
// natural [N1][N2][N3] <-> permuted [N3][xp][yp]
hipError_t launch_permute_real(const Plane &pl, const int *px, const int *py, const double *in, double *out,
                               hipStream_t st);
hipError_t launch_permute_complex(const Plane &pl, const int *px, const int *py, const double2 *in, double2 *out,
                                  int inverse, hipStream_t st);
// PZ81 LDA kernel f_xc(rho) (Ha bohr^3), zero where rho < 1e-10.
hipError_t launch_fxc(const double *rho, double *fxc, long n, hipStream_t st);
// Spin-polarized LSDA kernel from rho_up, rho_dn: fxc[0..2][i] = f_uu, f_ud, f_dd.
hipError_t launch_fxc_spin(const double *rho_up, const double *rho_dn, double *fxc, long n, hipStream_t st);

// proj:   Cpart -> C[k][m][v] = row_scale[m] * gscale * sum_G conj(T_e[m0+m][G]) X[k*nb+v][G]
hipError_t launch_zproj(const KPair *kp, int use_kq, int nk, const double2 *T, long t_stride, int m0, int M,
                        const double2 *X, int ld, int nb, const int *npw_of, double2 *Cpart, int nsplit,
                        const int *active, int tile, hipStream_t st);
hipError_t launch_zproj_reduce(int nk, int M, int nb, int nsplit, const double2 *Cpart, const double *row_scale,
                               double gscale, double2 *C, hipStream_t st);
// expand: Y[k*nb+v][G] += cscale * sum_m T_e[m0+m][G] C[k*c_kstride + m*nb + v]
hipError_t launch_zexpand(const KPair *kp, int use_kq, int nk, const double2 *T, long t_stride, int m0, int M,
                          const double2 *C, long c_kstride, double cscale, double2 *Y, int ld, int nb,
                          const int *npw_of, int npw_max, const int *active, int bv, hipStream_t st);
// tile (projection): workgroup tile 0 = 32x32, 1 = 64 rows x 32 bands, 2 = 32 x 64, 3 = 64 x 64;
// bv (expansion): 32 bv bands x 64 plane waves per workgroup, bv in {1, 2, 4}.
// The GEMMs' `active` argument (nullable) is a band map from launch_active_map: the tiles
// then cover only the active bands of each k, packed (outputs of other bands untouched).
// bmap[k][0] = active items of pair k, bmap[k][1 + j] = the band of the j-th ([nk][nb + 1]).
hipError_t launch_active_map(const int *active, int nk, int nb, int *bmap, hipStream_t st);
// preconditioned CG (one workgroup per item)
hipError_t launch_cg_init(const KPair *kp, int nb, int nitems, const double2 *B, double2 *Xv, double2 *R, double2 *P,
                          const double2 *AX, int have_x0, const double *diag, const double *eps, int ld,
                          const int *npw_of, long diag_stride, double *rz, double *bn, double *rn, int *active,
                          double tol, hipStream_t st);
hipError_t launch_cg_step(const KPair *kp, int nb, int nitems, double2 *Xv, double2 *R, double2 *P, const double2 *AP,
                          const double *diag, const double *eps, int ld, const int *npw_of, long diag_stride,
                          double *rz, const double *bn, double *rn, int *active, const double *tol, int *n_active,
                          int *n_bad, hipStream_t st);
// (tol is read from device memory, so a captured CG iteration serves every tolerance;
//  n_active / n_bad count the items still above tolerance / with a non-finite residual)
// FP32 variants (mixed-precision inner solves; scalars and reductions stay FP64).
hipError_t launch_zproj32(const KPair *kp, int use_kq, int nk, const float2 *T, long t_stride, int m0, int M,
                          const float2 *X, int ld, int nb, const int *npw_of, float2 *Cpart, int nsplit,
                          const int *active, int tile, hipStream_t st);
hipError_t launch_zproj_reduce32(int nk, int M, int nb, int nsplit, const float2 *Cpart, const double *row_scale,
                                 double gscale, float2 *C, hipStream_t st);
hipError_t launch_zexpand32(const KPair *kp, int use_kq, int nk, const float2 *T, long t_stride, int m0, int M,
                            const float2 *C, long c_kstride, double cscale, float2 *Y, int ld, int nb,
                            const int *npw_of, int npw_max, const int *active, int bv, hipStream_t st);
// BF16 variants (tables as packed bfloat16 complex, 32 bits each; vectors, outputs and
// accumulation FP32). tile: 0 = 32x32, 3 = 64x64 (others fall back to 32x32).
hipError_t launch_zproj16(const KPair *kp, int use_kq, int nk, const unsigned *T, long t_stride, int m0, int M,
                          const float2 *X, int ld, int nb, const int *npw_of, float2 *Cpart, int nsplit,
                          const int *active, int tile, hipStream_t st);
hipError_t launch_zexpand16(const KPair *kp, int use_kq, int nk, const unsigned *T, long t_stride, int m0, int M,
                            const float2 *C, long c_kstride, double cscale, float2 *Y, int ld, int nb,
                            const int *npw_of, int npw_max, const int *active, int bv, hipStream_t st);
// out[i] = bf16(re) | bf16(im) << 16, round to nearest even
hipError_t launch_to_bf16_pairs(const double2 *in, unsigned *out, long n, hipStream_t st);
hipError_t launch_cg_init32(const KPair *kp, int nb, int nitems, const float2 *B, float2 *Xv, float2 *R, float2 *P,
                            const double *diag, const double *eps, int ld, const int *npw_of, long diag_stride,
                            double *rz, double *bn, double *rn, int *active, double tol, const int *only,
                            const double *floor_abs, hipStream_t st);
hipError_t launch_cg_step32(const KPair *kp, int nb, int nitems, float2 *Xv, float2 *R, float2 *P, const float2 *AP,
                            const double *diag, const double *eps, int ld, const int *npw_of, long diag_stride,
                            double *rz, const double *bn, double *rn, int *active, const double *tol,
                            int *n_active, int *n_bad, const double *floor_abs, hipStream_t st);
// p[0..n) = v (a kernel, so that it can sit inside a captured graph)
hipError_t launch_fill_int(int *p, int n, int v, hipStream_t st);
hipError_t launch_fill_double(double *p, int n, double v, hipStream_t st);
// *p = device wall clock (constant rate, hipDeviceAttributeWallClockRate kHz)
hipError_t launch_clock_stamp(unsigned long long *p, hipStream_t st);
// R = B - AX (FP64; AX ignored when !have_x), R32 = (float) R, per-item norms and active flags.
hipError_t launch_residual64(const KPair *kp, int nb, int nitems, const double2 *B, const double2 *AX, int have_x,
                             double2 *R, float2 *R32, int ld, const int *npw_of, double *bn, double *rn, int *active,
                             double tol, int *count, double *floor_abs, hipStream_t st);
// (floor_abs, nullable: per-item absolute residual below which an inner solve stops)
// The same with A X from the FP32 operator (used where the FP32 operator is accurate enough).
hipError_t launch_residual64_ax32(const KPair *kp, int nb, int nitems, const double2 *B, const float2 *AX, double2 *R,
                                  float2 *R32, int ld, const int *npw_of, double *bn, double *rn, int *active,
                                  double tol, int *count, double *floor_abs, hipStream_t st);
// X (+)= (double) D for refined items.
hipError_t launch_refine_update(int nb, int nitems, double2 *X, const float2 *D, int ld, const int *refined,
                                int have_x, hipStream_t st);
hipError_t launch_to_f32(const double *in, float *out, long n, hipStream_t st);
// dn[s][m1][m2] = sum_k 2 w_k sum_v (B[k][5s+m1][v] conj(A[ek][5s+m2][v]) + (m1 <-> m2))
hipError_t launch_dn(const KPair *kp, int nk, int nh, int nb, const double2 *A, const double2 *B, double occ,
                     double2 *dn, hipStream_t st);
// mixing helpers
hipError_t launch_zdots(int nvec, const double2 *const *a, const double2 *b, long n, double2 *partial, double2 *out,
                        hipStream_t st);
hipError_t launch_zaxpy_list(long n, double2 *y, int nvec, const double2 *const *x, const double2 *coef,
                             hipStream_t st);
hipError_t launch_zsub(long n, const double2 *a, const double2 *b, double2 *out, hipStream_t st);
hipError_t launch_zscale_copy(long n, const double2 *a, double s, double2 *out, hipStream_t st);
// Load time.  dst[r][p] = src[r][order[p]] (p < npw; 0 up to ld) for r < nrows: a row-major
// [nrows][npw] table in the caller's plane-wave order to the internal stick order.
hipError_t launch_gather_rows(const double2 *src, int npw, const int *order, int nrows, double2 *dst, int ld,
                              hipStream_t st);
// dst[r][order[p]] = src[r][p] (p < npw): rows of length ld in the stick order to rows of
// length npw in the caller's order.
hipError_t launch_scatter_rows(const double2 *src, int ld, int npw, const int *order, int nrows, double2 *dst,
                               hipStream_t st);
// Jacobi diagonal of every entry e: kin + vmean[spin] + sum_r scale[r] |T_e[r]|^2 (1 on padding).
hipError_t launch_diag(const KPair *self, const EntryDev *ent, int n_entries, const double2 *T, long t_stride,
                       int nrows, const double *scale, const double *kin, const double *vmean, int ld, double *diag,
                       hipStream_t st);
// out[2b], out[2b+1] = sum and count of non-finite values of x[b*n .. b*n+n) (fixed order).
hipError_t launch_block_stats(const double *x, int nblocks, long n, double *out, hipStream_t st);
// x[i] *= s[i / per] for i < n: rows of `per` complex values scaled by one real each
// (the band occupations of right-hand-side rows, or the coefficients of a projection).
hipError_t launch_scale_rows(long n, long per, const double *s, double2 *x, hipStream_t st);

}  // namespace hp
