/*
 * pnof.h -- C ABI of the MI355X (gfx950) PNOF5 / PNOF7 / PNOF7s orbital-optimisation step.
 *
 * The operations follow M. Piris and I. Mitxelena, "DoNOF: an open-source implementation of
 * natural-orbital-functional-based methods for quantum chemistry", arXiv:2004.06142:
 *   energy          Section 2, Eqs. EPNOF7, Eg, Efg (PNOF5: Phi = 0; PNOF7s: Eq. Efg_s); multiplets of
 *                   highest multiplicity through N_I singly occupied orbitals (Eqs. intra, interab)
 *   J, K            Section 3.5, Eqs. JKpq and Gpmn (L = K for real orbitals, Section 2)
 *   Fock vectors    Section 3.2, Eqs. lowdin, Vee-s, Vee-d
 *   Lagrangian      Section 3.2, Eqs. lag and gval; symmetry criterion of Section 3.4
 *   orbital step    Section 3.2, Eq. Fockian, aufbau diagonal and zeta scaling; initial step of
 *                   Section 3.4 (diagonalisation of the symmetrised Lagrangian)
 *   ON maps         Section 3.1, Eqs. soo, sum1-h, woo (trigonometric), and a sigmoid map
 *
 * Conventions shared by every call
 *   - All array arguments are DEVICE pointers on the context's device, row-major, float64 unless
 *     stated.  The caller owns every buffer; the library never frees or retains them.
 *   - C[mu*nbf + p] = C_{mu p}: column p holds orbital p in the (orthonormal, S = I) AO basis.
 *   - n[p], p < nbf: per-spin occupation numbers; n[p] = 0 for p >= nact = npairs*(ncwo+1) + nsingle.
 *   - Orbital layout (fixed by npairs, ncwo, nsingle): the strong orbital of pair g is orbital g;
 *     the nsingle singly occupied orbitals of Omega_I (n = 1/2, each its own subspace, no
 *     intra-subspace term) are npairs .. npairs+nsingle-1; the ncwo weak orbitals of pair g are
 *     npairs + nsingle + ncwo*(npairs-1-g) + k, k = 0..ncwo-1 (consecutive blocks in reverse pair
 *     order, the coupling of the water tables of Section 5).
 *   - H: nbf x nbf symmetric one-electron matrix.
 *   - Two-electron integrals, by pnof_problem.ints:
 *       PNOF_INTS_ERI4_F64  ERI[((m*nbf + n)*nbf + l)*nbf + s] = (mn|ls), float64, nbf <= 64;
 *       PNOF_INTS_DF_F64    B[(P*nbf + m)*nbf + n], float64, (mn|ls) = sum_P B_Pmn B_Pls;
 *       PNOF_INTS_DF_BF16   the same B stored as bfloat16 (the stored values are exact inputs).
 *     B_P must be symmetric in (m, n).
 *   - Calls are asynchronous on the context's HIP stream; outputs are valid after that stream is
 *     synchronised.  Scalar outputs (E, max_asym) are device scalars.  Some steps also run on a
 *     second stream owned by the context (default priority): the orbital step's product of
 *     reflectors, and in the bf16-split density-fitted calls that form the Fock vectors the per-chunk
 *     D alpha, W diagonal and Y reduction.  That stream waits on an event recorded on the context's
 *     stream before its first use in a call, and the context's stream waits on its last event before
 *     the call's remaining work, so stream order as seen by the caller is unchanged.
 *   - Errors: arguments, shapes and enums are validated on the host before anything is enqueued;
 *     on error nothing is launched and the call returns a status; pnof_last_error() gives the text.
 *     A failed launch or an earlier asynchronous device error is returned as PNOF_E_DEVICE.
 *     Nothing throws across the ABI.
 *   - Workspace: device scratch comes from pnof_set_workspace (caller-owned, e.g. a torch tensor)
 *     when one of sufficient size has been set; otherwise the context allocates and keeps its own
 *     (grow-only, freed by pnof_destroy).
 *   - One context per host thread and stream; calls on one context must not overlap.
 */
#ifndef PNOF_H
#define PNOF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PNOF_ABI_VERSION 4

typedef struct pnof_ctx_s* pnof_ctx;

typedef enum {
  PNOF_OK = 0,
  PNOF_E_ARG = 1,          /* NULL pointer, bad context, bad scalar argument          */
  PNOF_E_SHAPE = 2,        /* inconsistent sizes                                        */
  PNOF_E_DTYPE = 3,        /* precision / integral kind combination not allowed        */
  PNOF_E_NOMEM = 4,        /* workspace allocation failed                               */
  PNOF_E_DEVICE = 5,       /* HIP launch or runtime error (possibly from an earlier call) */
  PNOF_E_NONFINITE = 6,    /* PNOF_CHECK_FINITE found a NaN / Inf in an input           */
  PNOF_E_UNSUPPORTED = 7,  /* valid request that the library does not implement       */
  PNOF_E_EIG = 8           /* the eigensolver did not converge                          */
} pnof_status;

typedef enum { PNOF5 = 5, PNOF7 = 7, PNOF7S = 8 } pnof_functional;

/* Arithmetic of the three-index contractions (X = B C, b = C^T X, Y = sum_P X W):
 *   PNOF_FP64        float64 matrix cores;
 *   PNOF_FP32        float32 matrix cores (v_mfma_f32_16x16x4f32): C, B, X and W rounded to float32,
 *                    float32 accumulation within a P row and over the rows of one P-split of Y, K in
 *                    float64, and the energy corrected to first order with 4 <Y_2e, C_A - float(C_A)>;
 *   PNOF_BF16        one bfloat16 pass per contraction, float32 accumulation (error study only);
 *   PNOF_BF16_SPLIT  16-bit matrix cores with float32 accumulation.  C_A is carried as a bf16 pair
 *                    C~ = hi + lo (|C - C~| <= 2^-17 |C|); X = B C~ takes 2 bf16 products against a
 *                    bf16 B.  X, W and C~ itself (for b) are carried as fp16 pairs of the value times
 *                    a power of two (about 22 significant bits) fixed per chunk of P rows from bounds
 *                    of |B| and |C|; b and Y take 3 fp16 products each (hi*hi, hi*lo, lo*hi).  A
 *                    float64 B is carried as an fp16 pair too (X then takes 3 fp16 products).  K sums
 *                    b^2 and Y its products in float32 over the rows of one P-split of one chunk,
 *                    then in float64; D and J = D^T D are float64.  The energy is corrected to first
 *                    order with 4 <Y_2e, C_A - C~> in float64.
 * Energies, lambda, J = D^T D, the eigensolver and all reductions are float64 in every mode. */
typedef enum { PNOF_FP64 = 0, PNOF_FP32 = 1, PNOF_BF16 = 2, PNOF_BF16_SPLIT = 3 } pnof_precision;

typedef enum { PNOF_INTS_ERI4_F64 = 0, PNOF_INTS_DF_F64 = 1, PNOF_INTS_DF_BF16 = 2 } pnof_ints;

enum { PNOF_CHECK_FINITE = 1 };

typedef struct {
  int32_t nbf;         /* AO basis size N_B                                   */
  int32_t naux;        /* density-fitting rank (0 for PNOF_INTS_ERI4_F64)     */
  int32_t npairs;      /* electron pairs N_II/2 (singlet: N_I = 0)            */
  int32_t ncwo;        /* weak orbitals per pair N_g (>= 1)                   */
  int32_t functional;  /* pnof_functional                                     */
  int32_t precision;   /* pnof_precision                                      */
  int32_t ints;        /* pnof_ints                                           */
  int32_t flags;       /* PNOF_CHECK_FINITE                                   */
  int32_t nsingle;     /* N_I singly occupied orbitals (multiplet S = N_I/2); 0: singlet */
} pnof_problem;

/* ---- context ---------------------------------------------------------------------------- */
/* Create a context on HIP device `device` issuing work on `hip_stream` (NULL = null stream). */
pnof_status pnof_create(pnof_ctx* out, int device, void* hip_stream);
void pnof_destroy(pnof_ctx ctx);
pnof_status pnof_set_stream(pnof_ctx ctx, void* hip_stream);
/* Text of the last error on this context (ctx may be NULL: the last error of this thread). */
const char* pnof_last_error(pnof_ctx ctx);
int pnof_abi_version(void);

/* Host-only validation of a problem description (no device access). */
pnof_status pnof_check_problem(const pnof_problem* prob);
/* Bytes of device workspace that the DF calls on `prob` use. */
pnof_status pnof_workspace_size(pnof_ctx ctx, const pnof_problem* prob, size_t* bytes);
/* Lend `bytes` of device memory at `dev` (256-byte aligned) to the context; NULL detaches. */
pnof_status pnof_set_workspace(pnof_ctx ctx, void* dev, size_t bytes);
/* Launch parameters of the density-fitted path (0 = automatic for every field):
 *   pchunk     rows of B processed per pass;
 *   nsplit_b   P-groups of the b / K contraction (each group keeps its own K partial sums);
 *   nsplit_y   P-groups of the Y contraction (each group keeps its own Y partial sums);
 *   x_variant, y_variant  block-tile shape of the bf16 X and Y contractions: 1 = 128 x 128 (two
 *              blocks per compute unit), 2 = 128 x 256 / 256 x 128, 3 = 256 x 256 with 8 waves
 *              (one block per compute unit).  Automatic: 3 when it pads the output no more than 128
 *              tiles do and both extents reach 512, else 1.  The float64 path ignores them.
 * Results do not depend on them beyond floating-point rounding order.  pnof_get_plan returns the
 * values a call on `prob` would use. */
typedef struct {
  int32_t pchunk, nsplit_b, nsplit_y, x_variant, y_variant;
} pnof_tuning;
pnof_status pnof_set_tuning(pnof_ctx ctx, const pnof_tuning* tuning);   /* NULL: all automatic */
pnof_status pnof_get_plan(pnof_ctx ctx, const pnof_problem* prob, pnof_tuning* out);
/* Shorthand for setting only pnof_tuning.pchunk. */
pnof_status pnof_set_pchunk(pnof_ctx ctx, int32_t pchunk);
/* Bind the integrals of repeated calls (Section 3.4: they stay fixed through an orbital
 * optimisation).  In the bf16 split mode every call otherwise reads all of B once more before its
 * contractions, for the row bounds of each chunk of P rows that fix the fp16 pairs' power-of-two
 * scales; pnof_bind_integrals makes that pass once, for `prob` under the current launch plan, and
 * keeps the bounds in the context.  A later call whose problem has the same nbf, naux and integral
 * kind, whose plan has the same pchunk and whose `ints` is the same device pointer reuses them; any
 * other call computes its own as before.  The caller must not change the bound integrals: after a
 * change, bind again (or unbind).  prob == NULL or ints == NULL unbinds.  Other precisions: nothing
 * to keep (PNOF_OK).  Allocates a few bytes per chunk once; later calls allocate nothing. */
pnof_status pnof_bind_integrals(pnof_ctx ctx, const pnof_problem* prob, const void* ints);

/* Measurement: between pnof_profile_begin and pnof_profile_end every launch of the three-index
 * contraction kernels (and of the eigensolver) is bracketed by HIP events recorded on the context
 * stream.  pnof_profile_end synchronises the stream and returns, per stage, the summed event time
 * in milliseconds and the number of launches (arrays of PNOF_NSTAGES entries). */
enum { PNOF_STAGE_X = 0, PNOF_STAGE_B = 1, PNOF_STAGE_Y = 2, PNOF_STAGE_EIG = 3, PNOF_NSTAGES = 4 };
pnof_status pnof_profile_begin(pnof_ctx ctx);
pnof_status pnof_profile_end(pnof_ctx ctx, double* ms, int64_t* launches);

/* ---- occupation numbers (Section 3.1) ------------------------------------------------------- */
/* kind 0, sigmoid-normalised: n_p = s(gamma_p) / sum_{r in pair(p)} s(gamma_r), ngamma = nact
 *   (the entries of singly occupied orbitals are not used).
 * kind 1, trigonometric (Eqs. soo, woo): ngamma = npairs*ncwo; gamma[g] is the strong orbital's
 *   variable of pair g and gamma[npairs + g*(ncwo-1) + i] the i-th weak one.
 * Singly occupied orbitals get n = 1/2.  n: nact outputs.  dn_dgamma: optional nact x ngamma
 * dense Jacobian (NULL to skip). */
pnof_status pnof_on_map(pnof_ctx ctx, int32_t kind, int32_t npairs, int32_t ncwo, int32_t nsingle,
                        const double* gamma, double* n, double* dn_dgamma);
/* Adjoint of the ON map: dEdgamma[r] = sum_p dEdn[p] dn_p/dgamma_r (ngamma outputs). */
pnof_status pnof_on_map_vjp(pnof_ctx ctx, int32_t kind, int32_t npairs, int32_t ncwo, int32_t nsingle,
                            const double* gamma, const double* dEdn, double* dEdgamma);

/* ---- NO integrals (Eqs. JKpq, Gpmn) --------------------------------------------------------- */
/* J, K: nact x nact, J_pq = (pp|qq), K_pq = (pq|pq).
 * Jq_ao, Kq_ao (optional, both NULL or both set): nq x nbf x nbf per-orbital AO matrices
 * J^q, K^q for the orbitals q_idx[0..nq) (device int32, each < nact). */
pnof_status pnof_jk(pnof_ctx ctx, const pnof_problem* prob, const double* C, const void* ints,
                    double* J, double* K, double* Jq_ao, double* Kq_ao, const int32_t* q_idx,
                    int32_t nq);

/* ---- energy (Eqs. EPNOF7, Eg, Efg) ---------------------------------------------------------- */
pnof_status pnof_energy(pnof_ctx ctx, const pnof_problem* prob, const double* C, const double* n,
                        const double* H, const void* ints, double* E);

/* ---- generalised Fock (Eqs. lowdin, Vee-s, Vee-d) -------------------------------------------- */
/* Y: nbf x nact, Y[:, q] = F^q c_q with F^q = n_q H + sum_r (alpha_qr J^r + beta_qr K^r) (the
 * paper's operator divided by 4).  Fq_ao (optional): nq x nbf x nbf matrices F^q, q in q_idx. */
pnof_status pnof_fock(pnof_ctx ctx, const pnof_problem* prob, const double* C, const double* n,
                      const double* H, const void* ints, double* Y, double* Fq_ao,
                      const int32_t* q_idx, int32_t nq);

/* ---- Lagrangian and gradients (Eqs. lag, gval, lowdin) ---------------------------------------- */
/* lambda: nbf x nbf, lambda_pq = c_p^T F^q c_q for q < nact, 0 for q >= nact.  E: energy.
 * Optional (NULL to skip): dEdC (nbf x nbf, = 4 F^q c_q, 0 for inactive columns), dEdn (nact),
 * max_asym (max |lambda_pq - lambda_qp|), J and K (nact x nact). */
pnof_status pnof_lagrangian(pnof_ctx ctx, const pnof_problem* prob, const double* C,
                            const double* n, const double* H, const void* ints, double* lambda,
                            double* E, double* dEdC, double* dEdn, double* max_asym, double* J,
                            double* K);

/* ---- without device allocation -------------------------------------------------------------- */
/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): pnof_lagrangian with the same arguments and results, its
 * workspace taken from a static device array of PNOF_STATIC_SCRATCH_BYTES on each GPU (held until
 * the process ends; pnof_create takes its address on the context's device).  Nothing is allocated:
 * no hipMalloc / hipFree, no rocBLAS (the float64 products run on the library's own GEMM), no second
 * stream (every step runs in order on the context's stream).  The rows of B per chunk are lowered
 * until the workspace fits the array; a problem that does not fit even with one row per chunk
 * returns PNOF_E_UNSUPPORTED, naming the bytes it needs.  All calls on one GPU share the array,
 * which keeps the last call's contents (each call clears what must start at zero): calls that
 * overlap on one GPU, from any context or stream, race. */
#define PNOF_STATIC_SCRATCH_BYTES (64u << 20)
pnof_status pnof_lagrangian_noalloc(pnof_ctx ctx, const pnof_problem* prob, const double* C, const double* n,
                                    const double* H, const void* ints, double* lambda, double* E, double* dEdC,
                                    double* dEdn, double* max_asym, double* J, double* K);

/* ---- orbital step (Eq. Fockian; Section 3.4) ------------------------------------------------ */
/* diag_prev == NULL: S = (lambda + lambda^T)/2.  Otherwise S_pq = lambda_qp - lambda_pq for p < q
 * (mirrored; the orientation of Eq. Fockian for which the first-order energy change of Eq. ene1
 * is negative when diag_prev increases with the index), S_pp = diag_prev[p], and when zeta > 0
 * every off-diagonal |S_pq| > zeta is divided by ten until it is <= zeta.  (eps, U) = eigh(S) in float64, eps ascending, each column of U
 * signed so that its largest-magnitude entry (lowest index on ties) is positive;
 * C_new = C U.  lambda, C, C_new: nbf x nbf; eps: nbf; S_out (optional): the matrix diagonalised.
 * C_new must not alias C or lambda.  The Householder reduction to tridiagonal form runs on the
 * library's kernels (one launch per column); the library's divide-and-conquer solver solves the
 * tridiagonal problem while a second stream of the context (default priority, forked and joined
 * with events) forms the product of the reflectors in blocks of 128; the eigenvectors are then that
 * product times the tridiagonal solver's.  nbf < 3 or nbf > 2048 use rocSOLVER's dsyevd.  Scratch:
 * about 9 nbf^2 doubles from the context's workspace (grown by the context if the lent one is
 * smaller).  PNOF_E_EIG if a secular equation of the tridiagonal solver does not converge. */
pnof_status pnof_orbital_step(pnof_ctx ctx, int32_t nbf, const double* lambda, const double* C,
                              const double* diag_prev, double zeta, double* C_new, double* eps,
                              double* S_out);

/* ---- NOF-MP2 reference terms (Section 4, Eqs. HFL and Esta) ----------------------------------- */
/* E_hf: Hartree-Fock-like energy of the natural orbitals, sum_g 2 A_g H_gg + sum_fg A_f A_g
 * (2 J_fg - K_fg) - sum_{g single} J_gg / 4 over the N_Omega = npairs + nsingle subspace-defining
 * orbitals (A = 1 strong, 1/2 single).  E_sta: static correlation,
 * sum_g sum_{p != q in Omega_g} sqrt(Lambda_p Lambda_q) Pi_qp K_pq - 4 sum_{f != g} sum_{p in
 * Omega_f, q in Omega_g} Phi_q^2 Phi_p^2 K_pq with Lambda_p = 1 - |1 - 2 n_p| and Pi of Eq. intra.
 * The dynamic term E^dyn needs amplitude equations that the paper does not give and is not
 * provided.  C, H: nbf x nbf; n: nact; E_hf, E_sta: device scalars.  Runs the J/K contractions
 * of pnof_jk on (C, ints). */
pnof_status pnof_nofmp2_terms(pnof_ctx ctx, const pnof_problem* prob, const double* C, const double* n,
                              const double* H, const void* ints, double* E_hf, double* E_sta);

/* ---- occupation optimisation at fixed orbitals (Section 3.1) --------------------------------- */
/* Minimises E(n(gamma)) = 2 sum_p n_p H_pp + sum_pq (alpha_pq J_pq + beta_pq K_pq) over the
 * unconstrained variables gamma of ON map `kind` (see pnof_on_map) with limited-memory BFGS
 * (backtracking line search with the Armijo condition).  Only H_pp = c_p^T H c_p, J and K of the
 * fixed orbitals enter: the integral transformation is done once per occupation optimisation.
 * C, H: nbf x nbf (H_pp is formed here); J, K: nact x nact from pnof_jk or pnof_lagrangian;
 * gamma: device, ngamma entries, the starting point on input and the minimiser on output.
 * E (host): final energy; iterations (host, optional).  The call synchronises the stream. */
typedef struct {
  int32_t maxiter;   /* <= 0: 1000 */
  int32_t memory;    /* correction pairs; <= 0: 10 */
  double gtol;       /* stop when max |dE/dgamma| <= gtol; <= 0: 1e-9 */
} pnof_on_opts;
pnof_status pnof_optimize_on(pnof_ctx ctx, const pnof_problem* prob, int32_t kind, const double* C,
                             const double* H, const double* J, const double* K, double* gamma,
                             const pnof_on_opts* opts, double* E, int32_t* iterations);

/* ---- orbital + occupation optimisation (Section 3.4) ------------------------------------------ */
/* The computational procedure of Section 3.4 on the device:
 *   initial step: occupations for the guess orbitals, then one diagonalisation of the symmetrised
 *     Lagrangian, whose eigenvalues are the first diagonal of the matrix of Eq. Fockian;
 *   iteration j: occupations for the orbitals phi^j (pnof_optimize_on); the matrix of Eq. Fockian
 *     (pnof_orbital_step conventions) with the previous eigenvalues on the diagonal and the zeta
 *     scaling; optionally DIIS over the last ndiis matrices (Section 3.3; matrices and error
 *     vectors, the off-diagonal elements, combined in the fixed AO basis); diagonalisation, new
 *     orbitals phi^{j+1} = phi^j U and new diagonal.
 * Stops when max |lambda_pq - lambda_qp| < delta (converged = 1), or when the three energy
 * differences of Section 3.4 fall below eps_n, eps_phi and eps (converged = 0), or after maxit
 * iterations.  C (in/out, nbf x nbf, orthonormal columns); gamma (in/out, ngamma) unless fix_n;
 * n (nact): the fixed occupations on input when fix_n, the final occupations on output otherwise.
 * Allocates its own device buffers for the duration of the call and synchronises the stream. */
typedef struct {
  int32_t on_kind;   /* ON map of the occupation optimisation (0 sigmoid, 1 trigonometric)   */
  int32_t maxit;     /* macro-iterations; <= 0: 200                                         */
  int32_t ndiis;     /* DIIS history; 0 or 1: off                                           */
  int32_t fix_n;     /* 1: occupations fixed at n (e.g. the Hartree-Fock limit)             */
  double eps_n, eps_phi, eps, delta, zeta;
  pnof_on_opts on;
} pnof_opt_opts;
typedef struct {
  double E, max_asym, d_n, d_phi, d_E;
  int32_t iterations, converged;
} pnof_opt_result;
pnof_status pnof_optimize(pnof_ctx ctx, const pnof_problem* prob, const double* H, const void* ints,
                          double* C, double* gamma, double* n, const pnof_opt_opts* opts,
                          pnof_opt_result* result);

/* ---- batches of independent problems (a potential-energy-surface scan) ---------------------- */
/* A batch runs the Lagrangian step (as pnof_lagrangian: E, lambda, optional dE/dC, dE/dn, max
 * asymmetry, and dE/dgamma through the ON map) for ninst independent problems of different sizes.
 * Two forms of one step:
 *   - a fixed sequence of grouped launches: every launch covers all instances, so small instances
 *     share the chip instead of each leaving it mostly idle (pnof_batch_info gives the count);
 *   - PNOF_BATCH_PERSISTENT: one persistent launch (after a launch that clears its scheduling
 *     state).  Its blocks claim work items of each instance's current phase -- the next phase of an
 *     instance opens when every item of the previous one is complete -- in instance order, so an
 *     instance completes as soon as its own work does; each instance's completion time is recorded
 *     on the device clock (pnof_batch_times).  The X and Y tile widths in use apply; b runs 64-wide.
 *     Each instance runs on one accelerator die (one L2): instances are spread over the device's
 *     dies by their work on the host, and a block serves the die it runs on.  A block that finds
 *     nothing to claim polls; once the batch's stall time (pnof_batch_set_stall) passes with no
 *     work item completed anywhere, it raises a stall flag and every block exits
 *     (pnof_batch_times then reports PNOF_E_DEVICE; so it does if the device's die ids do not map
 *     one to one onto its die count).  Split precision only.
 * Restrictions: every problem uses PNOF_INTS_DF_BF16 and the same precision (PNOF_BF16_SPLIT or
 * PNOF_BF16), flags == 0, and each instance's packed B and tile buffers stay below 2 GiB (roughly
 * nbf <= 600 at naux = 4 nbf); the functional may differ.
 *
 * pnof_batch_plan: validates the problems and allocates the batch's device workspace (owned by the
 *   batch, freed by pnof_batch_destroy; the only allocation of a batch).  Uses the context's device
 *   and stream; the context must outlive the batch.
 * pnof_batch_bind: io[i] gives instance i's device buffers (the pnof_lagrangian conventions:
 *   C, H, lambda, dEdC nbf x nbf; n, dEdn nbf; E and max_asym one double each; gamma and dEdgamma
 *   the variables of ON map on_kind, see pnof_on_map -- dEdgamma needs dEdn).  Binding copies every
 *   instance's B into the batch's padded layout (rows padded to a multiple of 32) and clears the
 *   tile workspace, on the context stream; later runs read that copy, so bind again after B
 *   changes.  C, n, H and gamma are read by every run at the bound addresses.
 * pnof_batch_run: enqueues one step of every instance on the context stream; flags:
 *   PNOF_BATCH_GRAPH captures the launches into a HIP graph on first use (on a private stream) and
 *   replays it afterwards (rebinding discards the graph); PNOF_BATCH_PERSISTENT selects the
 *   persistent form.  Runs on one batch must not overlap.
 * pnof_batch_times: after a persistent run, synchronises the context stream and writes each
 *   instance's completion time in microseconds after the run's start (us: ninst host doubles).
 *   (ABI version 4: gamma, dEdgamma, on_kind; run flags; completion times; stall time.) */
enum { PNOF_BATCH_GRAPH = 1, PNOF_BATCH_PERSISTENT = 2 };
typedef struct pnof_batch_s* pnof_batch;
typedef struct {
  const double* C;
  const double* n;
  const double* H;
  const void* ints;     /* B: naux x nbf x nbf bfloat16 */
  double* lambda;       /* required */
  double* E;            /* required: one device double */
  double* dEdC;         /* optional */
  double* dEdn;         /* optional (entries >= nact untouched) */
  double* max_asym;     /* optional: one device double */
  const double* gamma;  /* optional: ON-map variables of n (for dEdgamma) */
  double* dEdgamma;     /* optional: needs gamma and dEdn */
  int32_t on_kind;      /* ON map of gamma: 0 sigmoid, 1 trigonometric */
} pnof_batch_io;
pnof_status pnof_batch_plan(pnof_ctx ctx, int32_t ninst, const pnof_problem* probs, pnof_batch* out);
pnof_status pnof_batch_bind(pnof_batch batch, const pnof_batch_io* io);
pnof_status pnof_batch_run(pnof_batch batch, int32_t flags);
pnof_status pnof_batch_times(pnof_batch batch, double* us);
/* Time (device clock, microseconds) a persistent run may pass with no work item completed anywhere
 * before its blocks give up (0: the default, one second; at most 1e9). */
pnof_status pnof_batch_set_stall(pnof_batch batch, double microseconds);
/* Number of die groups the persistent form spreads the instances over (0: the device's XCC count,
 * the default; at most 16).  A block on die d serves group d mod dies; a count under which two dies
 * of the device share a group makes persistent runs stop early (pnof_batch_times reports
 * PNOF_E_DEVICE).  For testing and for partitioned devices whose count the runtime misreports. */
pnof_status pnof_batch_set_dies(pnof_batch batch, int32_t dies);
/* Device bytes held by the batch, and the number of launches one run enqueues. */
pnof_status pnof_batch_info(pnof_batch batch, size_t* bytes, int32_t* launches);
/* Tile widths along the active orbitals of the grouped X, b and Y contractions: 64 or 128, 0 for
 * the automatic choice (64 when it cuts that stage's padded matrix-core work, summed over the
 * instances, by a quarter or more).  May be called before or after pnof_batch_bind; it discards a
 * captured graph.  Results do not depend on the widths beyond floating-point rounding order.
 * pnof_batch_get_tiles writes the three widths in use.  (ABI version 3.) */
pnof_status pnof_batch_set_tiles(pnof_batch batch, int32_t x_tile, int32_t b_tile, int32_t y_tile);
pnof_status pnof_batch_get_tiles(pnof_batch batch, int32_t* tiles);
void pnof_batch_destroy(pnof_batch batch);

#ifdef __cplusplus
}
#endif
#endif /* PNOF_H */
