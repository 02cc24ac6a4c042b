/*
 * hp.h - C ABI of the MI355X Hubbard-response (DFPT) library.
 *
 * The library computes the linear response of the Hubbard-manifold occupations
 * of a periodic, norm-conserving insulator (spin-unpolarized, or collinear
 * spin-polarized with the same number of occupied states per spin) or metal
 * (unpolarized, cold smearing) to monochromatic
 * perturbations of those occupations, following Timrov, Marzari and
 * Cococcioni, "HP - A code for the calculation of Hubbard parameters using
 * density-functional perturbation theory":
 *   - the q-specific Sternheimer equation (Eq. 15) with the perturbing
 *     potential of Eq. 16 and the projectors of Eqs. 17-18,
 *   - the response occupations of Eq. 13 and the q-sum of Eq. 12,
 *   - the susceptibilities chi0, chi (Eq. 7) and U/V = chi0^-1 - chi^-1
 *     (Eqs. 8-9).
 *
 * Conventions (shared by every entry point):
 *   Units are Hartree atomic units.  The cell rows are the lattice vectors
 *   a1, a2, a3 (bohr); b = 2 pi inv(A)^T.  A plane wave of the basis at k is
 *   k + G with G = m . b for an integer Miller triple m; lattice-periodic
 *   functions are stored by coefficients c(G), u(r) = Omega^-1/2 sum_G c(G)
 *   e^{iG.r}.  Grid point (j1,j2,j3) is r = sum_i (j_i/N_i) a_i; Miller index
 *   m lands on grid index m mod N.  Real-space arrays are row-major
 *   [N1][N2][N3] (N3 fastest).  Complex arrays are interleaved (re, im) FP64.
 *   The projector tables are the lattice-periodic Bloch sums
 *   fbar_k(G) = Omega^-1/2 ftilde(k+G) e^{-i(k+G).tau}.
 *   nspin = 1 (closed shell): spin factor 2 in the occupations and densities.
 *   nspin = 2 (collinear spin-polarized): one electron per state, spin-resolved
 *   states, local potentials and densities; the perturbation of Eq. 16 acts on
 *   both spins, the response occupations are summed over spins (the site
 *   occupation of Eq. 7 is the trace over m and spin), and the Hxc response uses
 *   the LSDA kernel.
 *
 * Status codes: every call returns hp_status.  0 = success; > 0 = warning,
 * outputs written; < 0 = error, outputs untouched.  hp_last_error() gives a
 * thread-local message for the last non-zero status.  Argument checks run
 * before any GPU call, so argument errors are reported without a device.
 *
 * Ownership: input pointers are borrowed for the duration of a call only.
 * hp_ground_state_load copies everything it needs into device memory owned by
 * the returned context (from host memory, or device to device when
 * hp_ground_state.inputs_on_device = 1); outputs go to caller-allocated host
 * arrays.  A context
 * may be used by one host thread at a time; calls on one context are
 * serialized on its stream.
 */
#ifndef HP_H
#define HP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hp_status;

enum {
  HP_OK = 0,
  HP_WARN_NOT_CONVERGED = 1,  /* SCF or CG stopped at its iteration limit      */
  HP_ERR_ARG = -1,            /* NULL pointer, bad size or bad enum value       */
  HP_ERR_SHAPE = -2,          /* inconsistent shapes (sphere vs grid, k+q ...)  */
  HP_ERR_HIP = -3,            /* HIP runtime failure (message has the detail)   */
  HP_ERR_OOM = -4,            /* device allocation failed                       */
  HP_ERR_STATE = -5,          /* call not valid for the context's state         */
  HP_ERR_SINGULAR = -6,       /* chi0 or chi not invertible                     */
  HP_ERR_NUMERIC = -7         /* NaN or Inf met in an iterate                   */
};

enum { HP_FP64 = 0, HP_MIXED = 1 };   /* arithmetic of the Sternheimer solves */
/* Hubbard projectors: the given atomic d orbitals, or the ortho-atomic ones
 * phi~_i = sum_j (O^-1/2)_ji phi_j over every atomic orbital, O_ij = <phi_i|phi_j> (Eq. 6). */
enum { HP_PROJ_ATOMIC = 0, HP_PROJ_ORTHO_ATOMIC = 1 };
/* HP_MIXED: number type of the projection GEMMs inside the low-precision inner solves
 * (FP32 accumulation in every case; the FFTs and V_loc psi are FP32). */
enum { HP_GEMM_FP32 = 0, HP_GEMM_BF16 = 1, HP_GEMM_BF16_PV32 = 2 };
enum { HP_XC_LDA_PZ81 = 1 };          /* local xc kernel (Perdew-Zunger 1981)   */

/* One k-entry: a point of the Gamma-centred k mesh, or an extra k+q point.
 * The paper's ground-state hand-off (section "Ground-state calculation"):
 * occupied lattice-periodic states and energies at k and k+q. */
typedef struct hp_kpoint {
  uint32_t struct_size;   /* sizeof(hp_kpoint)                                     */
  double k_frac[3];       /* k in units of b                                       */
  double weight;          /* 1/N_k for mesh points, 0 for k+q-only entries         */
  int32_t npw;            /* number of plane waves of the sphere at k              */
  const int32_t *miller;  /* [npw][3] Miller indices (any order)                   */
  const double *eps;      /* [n_occ] occupied energies (Ha)                        */
  const double *u;        /* [n_occ][npw] complex, orthonormal rows                */
  const double *beta;     /* [n_beta][npw] complex, KB projector tables            */
  const double *phi;      /* [n_hub*5][npw] complex, Hubbard d orbitals, per site  */
  const double *atwfc;    /* HP_PROJ_ORTHO_ATOMIC: [n_atwfc][npw] complex, every   */
                          /* atomic orbital of the system; else may be NULL        */
} hp_kpoint;

/* The unperturbed ground state (paper: ground-state calculation section). */
typedef struct hp_ground_state {
  uint32_t struct_size;   /* sizeof(hp_ground_state)                               */
  double cell[3][3];      /* rows a1, a2, a3 (bohr)                                */
  int32_t fft[3];         /* N1, N2, N3: each a product of 2, 3 and 5, <= 256      */
  const double *v_loc;    /* [nspin][N1][N2][N3] total local KS potential (Ha)     */
  const double *rho0;     /* [nspin][N1][N2][N3] ground-state (spin) density        */
                          /* (electrons/bohr^3)                                    */
  int32_t n_occ;          /* occupied bands (the same at every k)                  */
  int32_t n_beta;         /* KB projectors                                         */
  int32_t n_hub;          /* Hubbard sites (5 d orbitals each)                     */
  const double *d_kb;     /* [n_beta] KB strengths (Ha)                            */
  const double *hub_tau;  /* [n_hub][3] Hubbard site positions (bohr)              */
  int32_t spin_factor;    /* electrons per state: 2 (nspin = 1) or 1 (nspin = 2)   */
  int32_t n_mesh;         /* the first n_mesh entries of each spin block form the  */
                          /* k mesh                                                */
  int32_t n_kpts;         /* total entries: nspin blocks of (mesh + extra k+q)     */
  const hp_kpoint *kpts;  /* [n_kpts]: spin-up block, then (nspin = 2) a spin-down */
                          /* block with the same k points and spheres in order     */
  int32_t xc;             /* HP_XC_LDA_PZ81                                        */
  int32_t inputs_on_device; /* 0: every array is host memory.  1: the bulk arrays    */
                          /* (v_loc, rho0 and, per entry, u, beta, phi, atwfc) are   */
                          /* device memory on the current device (e.g. torch tensors) */
                          /* and are copied device to device; the index and scalar   */
                          /* arrays the load plans from (kpts, miller, eps, d_kb,     */
                          /* hub_tau, hub_rows, hub_pot) stay host memory.  Host and  */
                          /* device inputs of equal values give identical contexts    */
                          /* (the same gathers and reductions run on the device).     */
                          /* The copies run on `stream`: the caller's writes to the   */
                          /* device arrays must be complete or ordered before it.     */
                          /* Other values: HP_ERR_ARG                                 */
  void *stream;           /* hipStream_t to run on, or NULL for a private stream   */
  int32_t projectors;     /* HP_PROJ_ATOMIC: phi as given; HP_PROJ_ORTHO_ATOMIC:   */
                          /* Loewdin-orthogonalized over all atomic orbitals (Eq. 6)*/
  int32_t n_atwfc;        /* HP_PROJ_ORTHO_ATOMIC: atomic orbitals per entry        */
  const int32_t *hub_rows;/* HP_PROJ_ORTHO_ATOMIC: [n_hub*5] row of atwfc that is d */
                          /* orbital m of Hubbard site s, at 5 s + m                */
  int32_t nspin;          /* 1 (unpolarized) or 2 (collinear spin-polarized)        */
  const double *hub_pot;  /* NULL, or [nspin][n_hub][5][5] complex Hermitian (Ha):   */
                          /* the ground-state Hubbard potential of Eq. 5 (on-site)  */
                          /* as the matrices M of sum_I sum_{m1 m2} M^I_{m1 m2}     */
                          /* |phi^I_m1><phi^I_m2| (e.g. U^I (delta/2 - n^I)), part  */
                          /* of the unperturbed Hamiltonian; its response is not     */
                          /* included (paper, after Eq. 10)                          */
  double degauss;         /* 0: insulator (n_occ fully occupied bands); > 0: metallic  */
                          /* ground state with cold (Marzari-Vanderbilt) smearing of  */
                          /* this width (Ha); n_occ is then the number of kept bands  */
                          /* (the first band above them must be empty and several     */
                          /* widths away); nspin must be 1                            */
  double efermi;          /* metallic: the Fermi energy (Ha)                         */
} hp_ground_state;

/* Convergence controls (the paper's inputhp keywords conv_thr_chi, niter_max,
 * alpha_mix, nmix; cg_tol plays the role of thresh_init for every iteration). */
typedef struct hp_scf_params {
  uint32_t struct_size;   /* sizeof(hp_scf_params)                                 */
  double conv_thr_chi;    /* stop when max_s |chi(q)_it - chi(q)_it-1| < this (1/Ha)*/
  double conv_thr_v;      /* ... and ||dV_out - dV_in|| / ||dV_out|| < this         */
  double cg_tol;          /* per-band ||r|| / ||b|| of every Sternheimer solve     */
  int32_t niter_max;      /* SCF iteration limit (paper default 100)               */
  double alpha_mix;       /* mixing factor (paper default 0.3)                     */
  int32_t nmix;           /* mixing history length (paper default 4), 1..8         */
  int32_t max_cg_iter;    /* CG iteration limit per solve                          */
  int32_t precision;      /* HP_FP64 or HP_MIXED                                   */
  int32_t verbosity;      /* 0 silent, 1 one line per SCF iteration on stderr      */
  double inner_tol;       /* HP_MIXED: relative tolerance of each FP32 inner solve */
  int32_t max_refine;     /* HP_MIXED: FP64 refinement rounds per solve (>= 1)      */
  int32_t graph_chunk;    /* 0: CG kernels launched one by one; 1..8: CG iterations  */
                          /* are captured once as hipGraphs of up to this many       */
                          /* iterations and replayed (same results, fewer launches   */
                          /* and host round trips)                                   */
  int32_t autotune;       /* 1: on first use of a launch shape, time the candidate    */
                          /* GEMM tiles / K splits and FFT plane batches on this      */
                          /* device and keep the fastest (cached in the context);    */
                          /* 0: fixed default shapes                                  */
  int32_t lowp_gemm;      /* HP_MIXED: HP_GEMM_FP32 (KB and alpha P_v GEMMs in FP32), */
                          /* HP_GEMM_BF16 (both in BF16), HP_GEMM_BF16_PV32 (KB in    */
                          /* BF16, alpha P_v in FP32).  Below BF16 accuracy every     */
                          /* solve is finished by FP64 residual refinement.          */
  int32_t find_atpert;    /* hp_response_matrix: 4 (or 0) perturb every site; 1      */
                          /* perturb one site per class of equal occupation trace    */
                          /* (within docc_thr, see hp_site_occupations) and rebuild  */
                          /* the other columns by comparing distances (dist_thr)     */
  double docc_thr;        /* find_atpert = 1: occupation-trace threshold (paper 5e-5) */
  double dist_thr;        /* find_atpert = 1: distance threshold (bohr, paper 6e-4)   */
  int32_t skip_equivalence_q; /* hp_response_matrix: 0 (paper default) solves only one */
                          /* q of each (q, -q) pair of the mesh and takes             */
                          /* chi(-q) = conj chi(q) (time reversal); 1 solves every q   */
  double lowp_trust_tol;  /* HP_MIXED, FP32 GEMMs: Sternheimer solves whose tolerance   */
                          /* is at or above this are finished in FP32 with no FP64     */
                          /* refinement, and their right-hand sides and response     */
                          /* density are formed in FP32 too (the adaptive SCF         */
                          /* tolerance of later iterations); 0 = the default 1e-6;    */
                          /* 1 or more refines every solve in FP64 (negative: error)  */
} hp_scf_params;

/* Statistics of one call (all fields written when the pointer is not NULL). */
typedef struct hp_scf_stats {
  uint32_t struct_size;   /* sizeof(hp_scf_stats), set by the caller               */
  int32_t scf_iters;      /* SCF iterations taken                                  */
  int32_t converged;      /* 1 if the SCF met both thresholds                      */
  int32_t cg_iters;       /* CG iterations summed over SCF iterations              */
  int64_t h_applies_fp64; /* single-band H applications in FP64                    */
  int64_t h_applies_lowp; /* single-band H applications in reduced precision       */
  double wall_s;          /* host wall time of the call                            */
  double chi_change;      /* last max |chi(q)_it - chi(q)_it-1|                     */
  double v_residual;      /* last ||dV_out - dV_in|| / ||dV_out||                   */
  double max_rel_resid;   /* largest final CG relative residual                    */
  double stage_s[8];      /* GPU time per stage: rhs, cg, drho, hxc, mix, dn, -, - */
} hp_scf_stats;

typedef struct hp_ctx hp_ctx;  /* opaque; owns every device buffer */

/* Copy the ground state to the GPU and precompute what every perturbation
 * reuses: the LDA kernel f_xc(rho0), plane-wave/grid maps, kinetic energies,
 * the shift alpha = 2 (max - min) of the occupied energies (text after
 * Eq. 18), the projections <phi_k|u_vk> and the real-space occupied states.
 * With HP_PROJ_ORTHO_ATOMIC the Hubbard projectors of every entry are first
 * built from its atomic orbitals: the overlaps O_k on the matrix cores, O_k^-1/2
 * on the host (Jacobi), the rows hub_rows of O_k^-1/2 applied on the matrix
 * cores (Eq. 6); phi is then not read.
 * With nspin = 2 the LSDA kernel (Perdew-Zunger interpolation between the
 * unpolarized and polarized fits) is built from the two spin densities.
 * With degauss > 0 (metals) the occupations f = occ((efermi - e)/degauss) of cold
 * smearing enter the Sternheimer right-hand side -(f_i - sum_j beta_ij |u_j><u_j|)
 * dV u_i, beta_ij = f_i theta_ij + f_j theta_ji + alpha theta_ji (f_i - f_j) /
 * (e_i - e_j), theta_ji = (1 + erf((e_j - e_i)/degauss))/2, and at q = 0 the
 * Fermi level shifts to keep the electron count (extra density and occupations
 * of the states at the Fermi level); the occupied-state density rho0 is then
 * sum_k w_k sum_i 2 f_ki |u_ki|^2 / Omega.
 * Errors: HP_ERR_ARG (NULL, bad sizes, nspin not 1 or 2, spin_factor != 3 - nspin,
 * spin blocks that differ in k points or spheres, xc unknown, bad projector settings), HP_ERR_SHAPE (sphere does not fit the grid, FFT size not
 * 2^a 3^b 5^c), HP_ERR_SINGULAR (linearly dependent atomic orbitals), HP_ERR_OOM,
 * HP_ERR_HIP.  On success *out owns all device memory. */
hp_status hp_ground_state_load(const hp_ground_state *gs, hp_ctx **out);

/* Self-consistent solution of Eq. 15 for a perturbation of Hubbard site
 * pert_site (0-based) at wavevector q (units of b), for every occupied band of
 * every mesh k (the entry holding k+q is found among the loaded entries,
 * modulo a reciprocal lattice vector).  Writes the response occupations of
 * Eq. 13 for every site s:
 *   dn0_out [n_hub][5][5] complex : after the first iteration (dV_Hxc = 0,
 *                                   the chi0 column of Eq. 7),
 *   dn_out  [n_hub][5][5] complex : at self-consistency (the chi column).
 * Index order [s][m1][m2]; Delta_q n^s_{m1 m2} is per Ha of perturbation and
 * includes the spin factor (nspin = 1) or the sum over both spins (nspin = 2).  Returns HP_WARN_NOT_CONVERGED when niter_max or
 * max_cg_iter was reached (outputs hold the last iterate), HP_ERR_SHAPE when a
 * k+q entry is missing, HP_ERR_NUMERIC on NaN/Inf. */
hp_status hp_sternheimer_scf(hp_ctx *c, int32_t pert_site, const double q_frac[3],
                             const hp_scf_params *p, double *dn0_out, double *dn_out,
                             hp_scf_stats *st);

/* chi0 and chi over the N_H * N_q sites of the q-supercell: runs
 * hp_sternheimer_scf for every site and every q of the Gamma-centred nq mesh
 * and sums with the phases of Eq. 12.  Site index = l * n_hub + s with l the
 * cell of the q-supercell (l1, l2, l3 lexicographic, l3 fastest).
 *   chi0_out, chi_out [(n_hub*Nq)^2] row-major real (1/Ha);
 *   max_imag_out      largest |imaginary part| dropped by the q-sum (may be NULL);
 *   st                accumulated statistics (may be NULL).
 * With p->find_atpert = 1 only one site per class of hp_site_occupations is
 * perturbed (at every q); each missing element chi[I][J] is copied from the
 * first computed chi[I2][J2] (J2, then I2 ascending) whose sites belong to the
 * classes of J and I, whose moments have the same relative sign (moments of
 * magnitude <= 1e-6 count as zero) and whose minimum-image distance in the
 * q-supercell differs from d(I, J) by at most p->dist_thr; HP_ERR_ARG if some
 * element has no such match.  The copy is exact when equal-distance pairs are
 * related by a symmetry of the crystal.  Unless p->skip_equivalence_q, a q point
 * whose -q partner (modulo a reciprocal vector) comes earlier in the mesh is not
 * solved: chi(-q)_{s s'} = conj chi(q)_{s s'} (time reversal).
 * Status as hp_sternheimer_scf (the worst over all pairs). */
hp_status hp_response_matrix(hp_ctx *c, const int32_t nq[3], const hp_scf_params *p,
                             double *chi0_out, double *chi_out, double *max_imag_out,
                             hp_scf_stats *st);

/* Ground-state occupation of every Hubbard site (Eq. 3): trace_out[s] =
 * sum_spin Tr n^{s, spin}, moment_out[s] = Tr n^{s, up} - Tr n^{s, dn} (0 when
 * nspin = 1), and class_out[s] = the representative of s when sites whose
 * traces differ by less than docc_thr are equivalent (the paper's default search
 * for the atoms to perturb; a site joins the first earlier representative within
 * docc_thr).  Any output may be NULL. */
hp_status hp_site_occupations(hp_ctx *c, double docc_thr, double *trace_out, double *moment_out,
                              int32_t *class_out);

/* U/V matrix = chi0^-1 - chi^-1 (Eqs. 8-9): U on the diagonal, V off it (Ha).
 * chi0, chi, uv_out are [n][n] row-major host arrays, n >= 1.  FP64 LU with
 * partial pivoting; HP_ERR_SINGULAR when a pivot falls below 1e-14 times the
 * largest |entry|.  Host-only: needs no context and no GPU. */
hp_status hp_hubbard_params(int32_t n, const double *chi0, const double *chi, double *uv_out);

/* Nearest-neighbour pairs for the inter-site V of Eq. 9 in the periodic
 * supercell that the q mesh images (Eq. 12).  Sites are numbered as in
 * hp_response_matrix: site (s, l) -> l * n_hub + s, cell l enumerating the
 * nq[0] x nq[1] x nq[2] offsets R_l (last index fastest), at hub_tau[s] + R_l . cell.
 * For each primitive site I = s (cell 0), every other supercell site J whose
 * minimum-image distance (over translations of the supercell) is within
 * dist_thr (bohr) of I's smallest such distance is a nearest neighbour; the
 * pair's V is uv[I][J] of hp_hubbard_params.  cell: rows a1, a2, a3 (bohr);
 * hub_tau [n_hub][3] (bohr).  Writes up to max_pairs (I, J, distance) triples,
 * I ascending, then J ascending; *n_pairs = total found (HP_ERR_ARG if it
 * exceeds max_pairs, or for NULL pointers, n_hub < 1, nq < 1, dist_thr < 0).
 * Host-only: needs no context and no GPU. */
hp_status hp_neighbours(const double cell[9], int32_t n_hub, const double *hub_tau, const int32_t nq[3],
                        double dist_thr, int32_t max_pairs, int32_t *pair_i, int32_t *pair_j, double *dist,
                        int32_t *n_pairs);

/* Free every resource of the context.  NULL is accepted. */
void hp_destroy(hp_ctx *c);

/* Thread-local description of the last non-zero status (never NULL). */
const char *hp_last_error(void);

/* ---- Diagnostics: single steps of the path, for parity checks ------------ */

/* y = H_k x for n vectors on entry `entry` (index into kpts; kinetic + the
 * entry's spin's local potential on the grid + KB projectors; the operator of
 * Eq. 15 without the alpha shift).
 * x, y: [n][npw] complex host arrays in the caller's plane-wave order. */
hp_status hp_apply_h(hp_ctx *c, int32_t entry, int32_t n, const double *x, double *y);

/* y = H_k x as hp_apply_h, with the reduced-precision operator the mixed form's inner
 * solves use: x rounded to FP32, FP32 z-stick and plane transforms and V_loc psi (the
 * plane variant chosen for FP32), projections per lowp_gemm (HP_GEMM_FP32, HP_GEMM_BF16 or
 * HP_GEMM_BF16_PV32) with FP32 accumulation; y returned widened to FP64.  For parity checks
 * of those kernels (the mixed form's answers are FP64-refined, so they do not show the
 * operator's own accuracy). */
hp_status hp_apply_h_lowp(hp_ctx *c, int32_t entry, int32_t n, int32_t lowp_gemm, const double *x, double *y);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): hp_apply_h on device arrays, with every
 * intermediate buffer (the vectors in the internal plane-wave order, the z-stick data of the
 * FFT round trip, the projection partial sums) in a fixed workspace of
 * HP_NOALLOC_SCRATCH_BYTES that the library holds per GPU for the life of the process.  The
 * call allocates and frees nothing and does not synchronize: it enqueues its kernels on the
 * context's stream and returns; y is valid once that stream has reached this point.
 *   x, y: device arrays [n][npw] complex (the entry's plane-wave order as given at load),
 *         n >= 1 and at most HP_NOALLOC_SCRATCH_BYTES / per-vector bytes, where a vector
 *         takes 16 (2 ld + 2 N3 ns_pad + 17 n_beta) bytes (ld: the largest sphere rounded
 *         up to 64, ns_pad: the most z-sticks of any entry rounded up to 32); larger n is
 *         rejected with HP_ERR_ARG (the message gives the limit), other errors as
 *         hp_apply_h.  The results equal hp_apply_h's.
 * Every call on one GPU uses that GPU's one workspace: calls that overlap in time on the
 * same GPU (two host threads, or two streams) race and give wrong results; calls queued on
 * one stream are ordered and safe. */
#define HP_NOALLOC_SCRATCH_BYTES (32u << 20)
hp_status hp_apply_h_noalloc(hp_ctx *c, int32_t entry, int32_t n, const double *x, double *y);

/* One linear solve of Eq. 15 at mesh point mesh_k for every occupied band,
 * with a given response potential dv ([nspin][N1][N2][N3] complex host array, or
 * NULL for dV_Hxc = 0): du_out [n_occ][npw(k+q)] complex, in the plane-wave order
 * of the entry holding k+q.  mesh_k = spin * n_mesh + k, 0 <= k < n_mesh.  Uses p->cg_tol, p->max_cg_iter, p->precision. */
hp_status hp_solve_first_order(hp_ctx *c, int32_t pert_site, const double q_frac[3], int32_t mesh_k,
                               const double *dv, const hp_scf_params *p, double *du_out);

/* The library's local xc kernel (the one hp_ground_state_load builds from rho0;
 * Perdew-Zunger 1981 LDA, zero where the density is below 1e-10) evaluated on the
 * device at given densities.  nspin = 1: rho [n], fxc_out [n] (Ha bohr^3);
 * nspin = 2: rho [2][n] (up, down), fxc_out [3][n] (f_uu, f_ud, f_dd, the LSDA
 * kernel).  Host arrays; HP_ERR_ARG for NULL pointers, n < 1 or nspin not 1 or 2. */
hp_status hp_xc_kernel(int32_t nspin, int64_t n, const double *rho, double *fxc_out);

/* ---- Per-kernel timing ------------------------------------------------------
 * hp_profile_start enables and resets per-kernel GPU timing on the context's
 * stream (HIP events around each launch; inside CG iterations replayed from
 * hipGraphs, device-clock stamps written by one-thread kernels before and after
 * each timed kernel, since events recorded by graph nodes cannot be queried);
 * hp_profile_stop synchronizes, disables timing and writes up to `max` records
 * (kernel name, launches, summed GPU milliseconds).  *n_out receives the number
 * written. */
typedef struct hp_kernel_time {
  const char *name;       /* static string owned by the library */
  int64_t calls;
  double total_ms;
} hp_kernel_time;

hp_status hp_profile_start(hp_ctx *c);
hp_status hp_profile_stop(hp_ctx *c, hp_kernel_time *out, int32_t max, int32_t *n_out);

/* ---- Autotuner report --------------------------------------------------------
 * JSON text (NUL-terminated, into buf of len bytes) of the launch shapes the
 * autotuner chose in this context: per GEMM shape (precision, rows, batch) the
 * projection tile, K split and expansion band tile with the measured and the
 * default times (ms), per precision the chosen plane variant of the local-potential
 * FFT with every variant's time (-1: not available for the grid), and per precision the chosen
 * z-transform variants (see hp_set_stick_variant) with their times (-1: not available).  HP_ERR_ARG if buf is too small. */
hp_status hp_tuning_report(hp_ctx *c, char *buf, int32_t len);

/* Pin launch shapes instead of timing them (used when hp_scf_params.autotune = 1;
 * a pinned shape is never re-tuned).  GEMM shape key: prec (64, 32, or 16 for
 * BF16), rows of the projector table (n_beta + n_occ for H, n_occ for P_c,
 * n_beta for the BF16 KB part, 5 n_hub and 5 for the Hubbard terms), batch (mesh
 * points per launch, 1..n_mesh).  tile 0..3 (BF16: 0 or 3) =
 * projection workgroup tile 32x32, 64x32, 32x64, 64x64 (rows x bands); nsplit =
 * K split of the projection, 1..16; expand_bands = 32, 64 or 128 bands per
 * expansion workgroup.  Plane variant 0..3 of the local-potential FFT round trip
 * (0: one z plane per 256-thread workgroup, 1: two per 256, 2: two per 512, 3: one
 * plane with the twiddles read from global memory; 1-3 only for 72x45, 144x45 and
 * 30x24 planes, 1-2 only for even N3 with two planes fitting in LDS; 4, 5, 6: prec 32
 * only, whole lines in registers with LDS only for the two transposes, on 128, 192 or
 * 256 threads holding as many z planes as their lines fill, for 24x24, 30x24, 48x24,
 * 48x48, 72x45 and 144x45 planes).  Errors:
 * HP_ERR_ARG for values out of range or variants not available for the grid. */
hp_status hp_set_gemm_shape(hp_ctx *c, int32_t prec, int32_t rows, int32_t batch, int32_t tile, int32_t nsplit,
                            int32_t expand_bands);
hp_status hp_set_plane_variant(hp_ctx *c, int32_t prec, int32_t variant);
/* z-transform variants (inverse: sphere -> sticks, forward: sticks -> sphere):
 * 0 = a workgroup per 32 sticks, 1 = a thread per stick (N3 = 24 or 40 only), 2 = a thread
 * per stick with the workgroup's plane waves staged through LDS (N3 = 24 or 40, when the
 * plane waves of 256 sticks fit in 96 KB).  The three give identical results. */
hp_status hp_set_stick_variant(hp_ctx *c, int32_t prec, int32_t inverse_variant, int32_t forward_variant);

#ifdef __cplusplus
}
#endif
#endif /* HP_H */
