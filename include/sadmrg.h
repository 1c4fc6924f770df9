/*
 * libsadmrg -- spin-adapted two-site DMRG for ab initio quantum chemistry on
 * AMD Instinct MI355X (gfx950).  C ABI.
 *
 * Method: Wouters, Poelmans, Ayers, Van Neck, "CheMPS2: a free open-source
 * spin-adapted implementation of the density matrix renormalization group for
 * ab initio quantum chemistry" (arXiv:1312.2415).
 *   - MPS ansatz, canonical forms, effective Hamiltonian, Davidson, SVD and
 *     truncation, sweeping: section "DMRG for ab initio quantum chemistry".
 *   - complementary operators (one-body folding, bare renormalised operators,
 *     integral-weighted complementary operators, Hermitian-conjugate storage):
 *     section "Complementary operators".
 *   - SU(2) x U(1) x P symmetry, reduced tensors (eq. tensordecomp), singlet
 *     embedding, doublet operators (eqs. creaannih1/2), two-site object and
 *     its decomposition (eqs. TTtoS, StoTT, kappa): section "Symmetry-adapted
 *     DMRG".
 *   - user-facing objects (Hamiltonian, Problem, ConvergenceScheme, Solve):
 *     section "CheMPS2 library".
 *
 * Conventions shared by every call:
 *   - All pointers are HOST pointers unless a parameter says otherwise.
 *     Inputs are copied before the call returns; the caller keeps ownership.
 *   - Spins are passed doubled (twoS = 2S).  Point-group irreps are integers
 *     0..order-1 whose direct product is XOR (D2h in Cotton order
 *     Ag,B1g,B2g,B3g,Au,B1u,B2u,B3u; subgroups use the low bits).
 *   - Two-electron integrals are chemist (ij|kl), dense L^4, row-major, with
 *     the symmetry of a real two-body operator, (ij|kl) = (kl|ij) = (ji|lk)
 *     (real orbitals add (ij|kl) = (ji|kl): eightfold); the paper's
 *     physics-notation V_ijkl equals (ik|jl).
 *   - Every call returns a status: 0 on success, 1 = converged-with-warning
 *     (Davidson hit its iteration cap), negative on error:
 *       SADMRG_EINVAL   bad argument / shape / call order
 *       SADMRG_ESYMM    N, S, irrep inconsistent, or empty symmetry sector
 *       SADMRG_EINTEG   integrals not symmetric within tolerance, or NaN/Inf
 *       SADMRG_ENOMEM   device allocation failed
 *       SADMRG_EDEVICE  HIP runtime error
 *     sadmrg_last_error() returns a description of the last failure.
 *   - All device work is enqueued on the context's stream (default stream
 *     unless sadmrg_set_stream is called); calls that return host data
 *     synchronise that stream.  One context is used by one host thread.
 */
#ifndef SADMRG_H
#define SADMRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SADMRG_OK 0
#define SADMRG_WARN_NOT_CONVERGED 1
#define SADMRG_EINVAL (-1)
#define SADMRG_ESYMM (-2)
#define SADMRG_EINTEG (-3)
#define SADMRG_ENOMEM (-4)
#define SADMRG_EDEVICE (-5)

typedef struct sadmrg_ctx sadmrg_ctx;

/* Library version string (static storage). */
const char* sadmrg_version(void);

/* Create a context for L orbitals on HIP device `device`.
 * group_order: 1, 2, 4 or 8 (C1 .. D2h); orb_irrep[L]: irrep of each orbital
 * in lattice order.  The paper's Hamiltonian object (section "The Hamiltonian").
 * Errors: EINVAL (L < 2, bad order or irreps), EDEVICE. */
int sadmrg_create(sadmrg_ctx** out, int L, int group_order, const int* orb_irrep, int device);

/* Destroy a context and release all its device memory.  NULL is allowed. */
void sadmrg_destroy(sadmrg_ctx* ctx);

/* Device-memory hooks (for instance a framework's caching allocator).
 * alloc_fn(bytes, device, user) returns a device block of at least `bytes`
 * on `device`, or NULL when it cannot (the call then fails with ENOMEM after
 * the library has given back the blocks it keeps cached); free_fn(ptr,
 * bytes, device, user) takes back a block alloc_fn returned, with the same
 * size.  Every device allocation of the context goes through them (the
 * context caches freed blocks and hands them out again; the cache is
 * returned through free_fn when memory runs short and at sadmrg_destroy).
 * Blocks are used on the context's stream.  The callbacks may be called from
 * host threads the library starts inside a call, so they must be
 * thread-safe; they must not call back into the library.  Set them right
 * after sadmrg_create, before the context allocates (EINVAL otherwise); NULL,
 * NULL returns to hipMalloc / hipFree.  Errors: EINVAL (one callback without
 * the other, or device memory already held). */
typedef void* (*sadmrg_alloc_fn)(size_t bytes, int device, void* user);
typedef void (*sadmrg_free_fn)(void* ptr, size_t bytes, int device, void* user);
int sadmrg_set_allocator(sadmrg_ctx* ctx, sadmrg_alloc_fn alloc_fn, sadmrg_free_fn free_fn, void* user);

/* Use `hip_stream` (a hipStream_t, may be NULL for the default stream) for all
 * subsequent device work of this context. */
int sadmrg_set_stream(sadmrg_ctx* ctx, void* hip_stream);

/* Set E_const, one-body h[L*L] (row-major, symmetric) and two-body eri[L^4]
 * (chemist, row-major).  h = h^T, (ij|kl) = (kl|ij) = (ji|lk) and the
 * point-group selection rules are checked to within sym_tol (EINTEG on
 * failure). */
int sadmrg_set_integrals(sadmrg_ctx* ctx, double e_const, const double* h, const double* eri, double sym_tol);

/* Target symmetry sector: N electrons, total spin twoS/2, irrep (the paper's
 * Problem object).  N >= 2 is required by the one-body folding of the
 * complementary-operator construction (section "Complementary operators",
 * trick (a)).  Errors: ESYMM. */
int sadmrg_set_target(sadmrg_ctx* ctx, int N, int twoS, int irrep);

/* Davidson parameters: residual-norm tolerance, maximum subspace size (2..64)
 * and maximum iterations per micro-iteration. */
int sadmrg_set_davidson(sadmrg_ctx* ctx, double tol, int max_sub, int max_iter);

/* Precision of the sigma product (section "The effective Hamiltonian
 * equation": the eigenproblem solved at every micro-iteration).
 * mode 0: FP64 everywhere (default).
 * mode 1: the Davidson sigma products use FP32 copies of the operators and of
 *   psi with FP32 accumulation until the residual reaches max(tol, mixed_tol)
 *   or, once below 6e-6 |theta|, stops improving (10 % over four iterations:
 *   the FP32 rounding floor); orthogonalisation, Ritz problem and residuals
 *   stay FP64.  Then FP64 Davidson steps refine the vector (one by default,
 *   sadmrg_set_refinement): the subspace of the vector and its preconditioned
 *   FP64 residual, two FP64 sigma products for the first step and one for
 *   each further step; the reported energy of the micro-iteration is the
 *   lowest FP64 Ritz value and the refined vector goes on to the
 *   decomposition.
 * mode 2: as mode 1, but the Davidson sigma products are BF16x3 on the FP32
 *   copies: each value is split into hi = bf16(x) and lo = bf16(x - hi), a
 *   product is hi*hi + hi*lo + lo*hi on the BF16 matrix cores with FP32
 *   accumulation (relative error about 2^-16); the stall test uses that
 *   rounding level.
 * sadmrg_sigma uses the reduced products in modes 1 and 2.  SVD, truncation
 * and renormalisation stay FP64.  Errors: EINVAL. */
int sadmrg_set_precision(sadmrg_ctx* ctx, int mode, double mixed_tol);
/* Number of FP64 Davidson steps that refine the reduced-precision solution of
 * modes 1 and 2 (default 1, allowed 1..8).  Each step works on the subspace
 * of the current vector and its preconditioned FP64 residual and costs one
 * FP64 sigma product (plus one for the first step); the refinement stops
 * early when a step cannot move the vector.  Contexts swept together by
 * sadmrg_batch_sweep must share it.  Errors: EINVAL. */
int sadmrg_set_refinement(sadmrg_ctx* ctx, int steps);
/* Renormalised operators recomputed instead of stored (section
 * "Sweeping": a sweep needs the blocks on both sides of the current two
 * sites; the paper keeps them on disk).  interval = 0 (default): every
 * left and right block stays in device memory.  interval > 0: only the
 * blocks at bonds 0, L and multiples of `interval` are kept; any other block
 * is rebuilt from the nearest kept block and the MPS tensors (enlargement
 * and renormalisation) when a step or the energy adjoint needs it, kept
 * while the sweep works through that stretch, and dropped once it has
 * passed, so that about 2 L / interval + interval blocks are held instead
 * of L + 1.  Turns the kept enlargements off (sadmrg_set_enlarge_cache).
 * Results equal those with every block stored up to rounding.  Errors:
 * EINVAL (interval < 0). */
int sadmrg_set_block_checkpoints(sadmrg_ctx* ctx, int interval);
/* Block statistics since sadmrg_stats_reset: blocks rebuilt, host seconds
 * spent rebuilding them, the largest device bytes the blocks held at once,
 * and the number of blocks held now.  Pointers may be NULL. */
int sadmrg_stats_blocks(sadmrg_ctx* ctx, int64_t* rebuilt, double* seconds, double* max_bytes, int* held);

/* Davidson iterations replayed from a recorded launch sequence (section "The
 * effective Hamiltonian equation": the iterative eigensolver of every
 * micro-iteration).  replays = 0 (default): the host drives every
 * iteration.  replays > 0: after the first sigma product, one whole
 * iteration of every solve of the call (the lockstep solves of
 * sadmrg_batch_sweep included) -- Ritz pair, residual, convergence test,
 * preconditioned and orthogonalised correction, restart of a full subspace,
 * sigma product of the new vector and its row of the projected matrix -- is
 * recorded once per micro-iteration as a HIP graph that reads each solve's
 * subspace size and flags from device memory, and replayed `replays` times
 * between two host checks of those flags; a finished solve's kernels (its
 * GEMM passes included) return at once.  Results are those of the
 * host-driven iterations.  Not used on the legacy default stream (a null
 * stream set by sadmrg_set_stream) or for one-element problems.  Contexts
 * swept together by sadmrg_batch_sweep must share it.  Errors: EINVAL
 * (replays outside 0..64). */
int sadmrg_set_davidson_graph(sadmrg_ctx* ctx, int replays);
/* Counters of the recorded iterations since sadmrg_stats_reset: seconds of
 * the replayed segments (sigma products and every other step of them), host
 * seconds spent recording and instantiating the sequences (a batch's times
 * are split evenly over its contexts), the sigma flops and sigma products
 * inside the replays, replays and recordings.  Pointers may be NULL. */
int sadmrg_stats_graph(sadmrg_ctx* ctx, double* seconds, double* record_seconds, double* sigma_flops,
                       int64_t* sigma_calls, int64_t* replays, int64_t* records);

/* Precision of the renormalisation products (section "Sweeping": the new
 * block's operators U^T O U after every decomposition).  mode 0 (default):
 * FP64.  mode 1: FP32 copies of the enlarged operators (the sigma's FP32
 * copies when the step has them) and of the tensor, FP32 products and
 * accumulation, the new block stored in FP64.  mode 2: BF16x3 products on
 * those FP32 copies.  The rounding stays in the renormalised operators for
 * every later step and sweep.  Contexts swept together by
 * sadmrg_batch_sweep must share it.  Errors: EINVAL. */
int sadmrg_set_renorm_precision(sadmrg_ctx* ctx, int mode);

/* Residual target of that refinement (default 0: always the set number of
 * steps).  With tol > 0, steps after the first run only while the FP64
 * residual norm |H x - theta x| of the refined vector is above tol, up to
 * the number set by sadmrg_set_refinement; a reduced-precision phase that
 * stopped on its rounding floor (BF16x3 products) then gets the FP64 steps it
 * needs to reach the residual an FP64 solve would have.  Contexts swept
 * together by sadmrg_batch_sweep must share it.  Errors: EINVAL. */
int sadmrg_set_refinement_tol(sadmrg_ctx* ctx, double tol);

/* Seed of the counter-based generator used for the random initial MPS. */
int sadmrg_set_seed(sadmrg_ctx* ctx, uint64_t seed);

/* Create the initial MPS (section "DMRG" of the library description): the
 * bond dimension D is split equally over the symmetry sectors of every bond,
 * capped by the FCI dimension, and filled with random numbers; the tensors of
 * sites 1..L-1 are right-normalised and all right renormalised operators are
 * built.  Errors: ESYMM (empty sector), ENOMEM, EDEVICE. */
int sadmrg_init_mps(sadmrg_ctx* ctx, int D);

/* Run one macro-iteration (a left-to-right pass over i = 0..L-2 followed by a
 * right-to-left pass over i = L-2..0; section "Sweeping") keeping at most D
 * reduced states per bond.  *e_min receives the lowest energy of this
 * macro-iteration.  Returns 1 if some Davidson solve hit max_iter. */
int sadmrg_sweep(sadmrg_ctx* ctx, int D, double* e_min);

/* One macro-iteration (as sadmrg_sweep) of each of n independent problems,
 * run in lockstep: micro-iteration r of every context still sweeping, then
 * r + 1.  The paper treats each state of its carbon-dimer study as its own
 * calculation in its own symmetry sector (section "Bond dissociation
 * curves") and parallelises within a calculation over the sparse blocks
 * (section "DMRG" of the library description); here the sigma products of
 * all contexts in one Davidson iteration go out as one launch per GEMM pass,
 * the accumulating pass balanced over the whole batch.
 *   ctxs[n]: distinct contexts with an MPS, every centre at the left end
 *            (as after sadmrg_init_mps, sadmrg_mps_import or a sweep), all on
 *            one device and one stream (sadmrg_set_stream) and in one
 *            precision mode.  Sizes, sectors and schedules may differ.
 *   D[n]:    bond dimension of each context (host array).
 *   e_min[n] (may be NULL): lowest energy of each context's macro-iteration.
 *   stats[10] (may be NULL): seconds, algorithmic flops and number of the
 *            shared FP64 sigma launches, then the same for FP32 (zero for a
 *            batch of one, which runs as sadmrg_sweep); then the host wall
 *            seconds of the phases: step preparation, Davidson, FP64
 *            refinement (mixed precision), decomposition and update.
 * Each context's result equals its own sadmrg_sweep up to the summation
 * order of the shared launches.  Returns 1 if some Davidson solve hit
 * max_iter; on an error every context gets the message, and the contexts
 * are left mid-sweep (re-import or re-initialise them).  Errors: EINVAL,
 * ENOMEM, EDEVICE. */
int sadmrg_batch_sweep(sadmrg_ctx* const* ctxs, int n, const int* D, double* e_min, double* stats);

/* Tune the launch shape of the sigma product on the prepared step (call
 * after sadmrg_prepare_step; the paper's parallelisation over sparse blocks,
 * section "DMRG" of the library description, here as grouped GEMM launches).
 * Twelve candidate plans are timed, each over `reps` FP64 sigma calls on a
 * fixed pseudo-random vector: the first GEMM pass with one output tile per
 * workgroup or 8 cost-balanced ranges per compute unit, times the
 * accumulating pass with 12, 16, 24, 32, 48 or 64 ranges per compute unit
 * (defaults: one tile per workgroup, 64 ranges).  The fastest pair is kept
 * for this context (later steps are planned with it) and the step is
 * re-planned.  Results do not depend on the choice beyond the summation
 * order of cut tiles.  *gpc1, *gpc2 (may be NULL): the chosen pair (0 = one
 * tile per workgroup); table[36] (may be NULL): the candidates' pairs
 * (table[2c], table[2c+1]) and mean ms per sigma (table[24 + c]).  The
 * sigma statistics exclude the timing calls; the content of the step's
 * input vector is overwritten.  Errors: EINVAL (no prepared step, reps < 1),
 * ENOMEM, EDEVICE. */
int sadmrg_autotune(sadmrg_ctx* ctx, int reps, int* gpc1, int* gpc2, double* table);

/* Set the sigma plans' workgroups per compute unit directly (as
 * sadmrg_autotune would choose them): gpc1 for the first GEMM pass, gpc2 for
 * the accumulating pass, 0 = one output tile per workgroup, at most 64.
 * Takes effect from the next prepared step.  Errors: EINVAL. */
int sadmrg_set_launch_shape(sadmrg_ctx* ctx, int gpc1, int gpc2);

/* How each sigma product out += c op(A) psi op(C) picks its contraction
 * order (left first: T = op(A) psi, then T op(C); right first: U = psi
 * op(C), then op(A) U).  mode 0 (default): fewer flops.  mode 1: fewer bytes
 * streamed from memory when every 64-wide output tile reads its panels of
 * op(A), op(C) and the intermediate (the psi block stays in the caches),
 * flops deciding ties.  Results differ only by rounding.  Takes effect from
 * the next prepared step.  Errors: EINVAL. */
int sadmrg_set_contraction_order(sadmrg_ctx* ctx, int mode);

/* Workgroup order of the two sigma GEMM passes (1 = on, 0 = off, per pass).
 * The dispatcher deals the workgroups of a launch to the device's eight XCDs
 * in turn, and each XCD has its own L2 cache.  With the order on, the tiles
 * (or tile ranges) are split into eight contiguous parts and part x runs on
 * XCD x, so the tiles of one product, which read the same operand panels,
 * run on one XCD close in time.  Results do not depend on it.  Takes effect
 * from the next prepared step.  Errors: EINVAL. */
int sadmrg_set_xcd_order(sadmrg_ctx* ctx, int pass1, int pass2);

/* Free and total bytes of device memory on a device (the library's cached
 * blocks count as used).  Errors: EINVAL, EDEVICE. */
int sadmrg_device_memory(int device, size_t* free_bytes, size_t* total_bytes);

/* Keep enlarged blocks for the next pass (on = 1, the default) or build
 * every enlargement afresh (on = 0, which also releases the kept ones).  In a
 * left-to-right pass the right blocks are the ones the previous
 * right-to-left pass built (section "Sweeping"), so the enlargement of the
 * unchanged side at step i equals the one made there; results are identical
 * either way.  Kept blocks of all contexts of the process share a ceiling
 * of two fifths of the device memory; the oldest go first.  Errors: EINVAL. */
int sadmrg_set_enlarge_cache(sadmrg_ctx* ctx, int on);

/* Run a convergence scheme (section "Convergence scheme"): n instructions of
 * (D[i], e_conv[i], max_sweeps[i], noise[i]).  *e_min receives the lowest
 * variational energy over all micro-iterations (the paper's Solve).  With
 * noise[i] = gamma > 0, every decomposition adds gamma/2 * w * u_e to the
 * two-site object, w the largest discarded weight of the previous left- or
 * right-pass and u_e uniform in [-1, 1) from the counter generator keyed by
 * (seed, 0x4E4F << 40 | pass << 16 | step, element), passes counted from the
 * MPS's creation or import; the object's sign is first chosen so that its
 * inner product with u is non-negative.  noise may be NULL (no noise); negative noise is
 * EINVAL. */
int sadmrg_solve(sadmrg_ctx* ctx, int n, const int* D, const double* e_conv, const int* max_sweeps,
                 const double* noise, double* e_min);

/* Discarded-weight extrapolation (section "Extrapolation"): the energies of
 * a run with several D lie on E(D) = E0 + C1 w_disc(D) for small discarded
 * weights.  n pairs (w[i] >= 0, e[i]) give the least-squares line; a pair
 * with w = 0 is an exact energy at its D and is returned as E0 (the lowest of
 * them) with C1 = 0; a single truncated pair gives its energy and C1 = 0.
 * Host arithmetic only.  Errors: EINVAL (n < 1, null pointers, negative or
 * non-finite values). */
int sadmrg_extrapolate(int n, const double* w, const double* e, double* e0, double* c1);

/* A convergence scheme run stage by stage (each stage as sadmrg_solve with
 * one instruction), then the extrapolation above: E(D) of a stage is the
 * lowest energy of its last macro-iteration and w(D) that macro-iteration's
 * largest discarded weight.  points[3n] (may be NULL) receives (D, w, E) per
 * stage; *e0, *c1 (may be NULL) the fit.  Returns 1 if some Davidson solve
 * hit its iteration cap.  Errors: as sadmrg_solve. */
int sadmrg_solve_extrapolated(sadmrg_ctx* ctx, int n, const int* D, const double* e_conv, const int* max_sweeps,
                              const double* noise, double* points, double* e0, double* c1);

/* ------------------------------------------------------------------------
 * DMRG-SCF (section "DMRG-SCF" of the library description): orbital
 * optimisation of a complete-active-space wavefunction with this library's
 * DMRG as the active-space solver, by the augmented-Hessian Newton-Raphson
 * method with the exact Hessian.  Conventions: real orbitals, chemist
 * integrals g_pqrs = (pq|rs); D_pq = <E_pq>, d_pqrs = <E_pq E_rs - d_qr
 * E_ps> (= Gamma^A_{pr;qs}); E = e_nuc + sum h_pq D_pq + 1/2 sum g_pqrs
 * d_pqrs; an orbital update is phi'_p = sum_q phi_q R_qp with R = exp(-K),
 * K antisymmetric with parameters K_pq, p > q.  All host arithmetic.
 * ------------------------------------------------------------------------ */
/* h_out = R^T h R and eri_out_ijkl = sum_pqrs R_pi R_qj R_rk R_sl eri_pqrs
 * (L x L and L^4, row-major; R orthogonal, column j = new orbital j).
 * Errors: EINVAL, ENOMEM. */
int sadmrg_rotate_integrals(int L, const double* R, const double* h, const double* eri, double* h_out,
                            double* eri_out);
/* R = exp(kappa) for an antisymmetric L x L kappa (EINVAL if it is not
 * antisymmetric to 1e-12): Taylor series after scaling, repeated squaring,
 * columns re-orthonormalised. */
int sadmrg_rotation(int L, const double* kappa, double* R);
/* Orbital derivatives of E with the RDMs D[L*L], d[L^4] held fixed:
 * the generalised Fock matrix F_pq = sum_m D_pm h_qm + sum_mnt d_pmnt g_qmnt
 * (fock[L*L], may be NULL), the gradient dE/dK_pq = 2 (F_pq - F_qp) for the
 * npairs pairs (pairs[2a] = p > pairs[2a+1] = q) into grad[npairs], and, when
 * hess is not NULL, the exact Hessian into hess[npairs^2]:
 *   H_pq,rs = (1 - P_pq)(1 - P_rs) [2 D_pr h_qs - (F_pr + F_rp) d_qs + 2 Y_pqrs],
 *   Y_pqrs = sum_mn [(d_pmrn + d_pmnr) g_qmsn + d_prmn g_qsmn].
 * Errors: EINVAL (bad pair), ENOMEM. */
int sadmrg_orbital_derivatives(int L, const double* h, const double* eri, const double* D, const double* d,
                               int npairs, const int* pairs, double* grad, double* hess, double* fock);
/* The DMRG-SCF loop.  ctx is an active-space context: created with one
 * orbital per active orbital (in increasing full-space index order, with
 * their irreps) and its target set to the active electrons (N - 2 n_core),
 * spin and irrep; its Davidson and precision settings apply.  Full space:
 * Lt orbitals with irreps orb_irrep[Lt] and classes cls[Lt] (0 core =
 * doubly occupied, 1 active, 2 virtual), nuclear repulsion e_nuc, h[Lt^2],
 * eri[Lt^4] in the starting orbitals.  Each iteration: rotate the integrals
 * to the current orbitals; fold the core into the active Hamiltonian
 * (E_core = e_nuc + sum_c 2 h_cc + sum_cc' [2 (cc|c'c') - (cc'|c'c)],
 * h_tu + sum_c [2 (tu|cc) - (tc|cu)]); run the convergence scheme (n_sched
 * instructions as sadmrg_solve; the previous iteration's MPS is the start);
 * form gamma and Gamma^A (sadmrg_calc2dm) and the full-space D and d of the
 * closed-shell core times the active state; stop if the norm of the gradient
 * over the non-redundant rotations (p > q of different classes and the same
 * irrep) is below grad_tol; else take the augmented-Hessian step (lowest
 * eigenvector (v0, v) of [[0, g^T], [g, H]], x = v / v0, scaled to norm <=
 * max_step) and update R <- R exp(-K(x)).
 *   U[Lt*Lt] (may be NULL): in, the starting rotation (NULL: identity); out,
 *     the final one (columns = optimised orbitals in the starting basis).
 *   history[2*max_iter] (may be NULL): per iteration, the energy at that
 *     iteration's orbitals and the gradient norm.
 *   *n_iter, *energy (may be NULL): iterations run, last energy.
 * The gradient of the last iteration is below grad_tol unless *n_iter ==
 * max_iter.  Errors: EINVAL (arguments, active orbitals that do not match
 * the context), ESYMM (no target on the context), and those of sadmrg_solve. */
int sadmrg_dmrgscf(sadmrg_ctx* ctx, int Lt, const int* orb_irrep, const int* cls, double e_nuc, const double* h,
                   const double* eri, int n_sched, const int* D, const double* e_conv, const int* max_sweeps,
                   const double* noise, double grad_tol, int max_iter, double max_step, double* U,
                   double* history, int* n_iter, double* energy);

/* Excited states by projection (section "CheMPS2 library", the DMRG object:
 * newExcitation).  sadmrg_push_excitation keeps the current MPS as the state
 * Psi_k (normalised; it must have its two-site centre at the left end, as
 * after a sweep or an import there) with weight eta > 0; every later solve
 * of this context uses H_m = H_0 + sum_k eta_k |Psi_k><Psi_k|, which pushes
 * the lower states up by eta_k and so targets the next state of the same
 * (N, S, irrep) sector (eta must exceed the gap to it).  The current MPS is
 * left as it is: start the next state with sadmrg_init_mps or
 * sadmrg_mps_import.  On the two-site space the extra term is sum_k eta_k
 * <phi_k|x> phi_k with phi_k the projection of Psi_k, built from overlap
 * environments of the current and the stored MPS that follow the sweep;
 * sadmrg_sigma and sadmrg_heff_diagonal include it, the density matrices
 * (sadmrg_rdm, sadmrg_calc2dm) are those of the state for H_0.  At most 64
 * states; sadmrg_set_target removes them, sadmrg_clear_excitations too.
 * Errors: EINVAL (eta <= 0, centre not at the left end, too many states). */
int sadmrg_push_excitation(sadmrg_ctx* ctx, double eta);
int sadmrg_clear_excitations(sadmrg_ctx* ctx);

/* Energies: lowest over all micro-iterations so far, last micro-iteration's,
 * and the largest discarded weight of the last macro-iteration. */
int sadmrg_get_energy(sadmrg_ctx* ctx, double* e_min, double* e_last, double* wdisc_max);

/* Per-micro-iteration energies recorded so far (size query when out == NULL:
 * *n receives the count). */
int sadmrg_get_trace(sadmrg_ctx* ctx, double* out, int* n);

/* Spin-summed reduced density matrices of the current MPS (the paper's
 * calc2DM, section "CheMPS2 library", the DMRG object):
 *   Gamma^A_{ij;kl} = sum_{s t} <a+_{i s} a+_{j t} a_{l t} a_{k s}>,
 *   gamma_ij = sum_s <a+_{i s} a_{j s}> = sum_k Gamma^A_{ik;jk} / (N - 1),
 * evaluated at the current two-site centre (after a sweep, a micro-iteration
 * or an import) as the derivative of E = <psi|H|psi> (normalised two-site
 * object) with respect to the integrals, in reverse mode through every
 * complementary-operator construction and renormalisation of both blocks.
 * The blocking formulas keep each creator next to its own annihilator
 * partner in every integral they read, so the derivative is taken over
 * integrals with only the symmetry of a real two-body operator and Gamma^A
 * comes out whole, not symmetrised over (ik|jl) = (ki|jl).
 * rdm1[L*L] (row-major, may be NULL) and rdm2[L^4] (Gamma^A_{ij;kl} at
 * [i][j][k][l], may be NULL) are host arrays; *energy (may be NULL) receives
 * E = E_const + sum h_ij gamma_ij + 1/2 sum (ik|jl) Gamma^A_{ij;kl}.  Cost:
 * one reverse pass over the whole chain.  Errors: EINVAL (no two-site
 * centre), ESYMM (no target), ENOMEM. */
int sadmrg_rdm(sadmrg_ctx* ctx, double* rdm1, double* rdm2, double* energy);

/* All calc2DM outputs from one reverse pass (same definitions as sadmrg_rdm):
 *   gamma_a[L^4] (may be NULL): Gamma^A; layout 0 = paper order,
 *     gamma_a[i][j][k][l] = Gamma^A_{ij;kl}; layout 1 = chemist order,
 *     gamma_a[p][q][r][s] = Gamma^A_{pr;qs}, so that E = E_const +
 *     sum h_pq gamma_pq + 1/2 sum (pq|rs) gamma_a[p][q][r][s];
 *   gamma_b[L^4] (may be NULL, paper order): Gamma^B_{ij;kl} = sum_{s t}
 *     (-1)^(s-t) <a+_{i s} a+_{j t} a_{l t} a_{k s}> averaged over the 2S+1
 *     members of the multiplet (the singlet-embedding spin is traced out; a
 *     singlet has one member).  For that SU(2)-invariant average the spin
 *     structure fixes Gamma^B_{ij;kl} = -(Gamma^A_{ij;kl} + 2 Gamma^A_{ij;lk})/3;
 *   rdm1[L*L], *s2 = <S^2> = -N(N-4)/4 - 1/2 sum_ij Gamma^A_{ij;ji} and
 *     *energy (each may be NULL).
 * Errors: EINVAL (bad layout, no two-site centre), ESYMM, ENOMEM. */
int sadmrg_calc2dm(sadmrg_ctx* ctx, double* gamma_a, double* gamma_b, int layout, double* rdm1, double* s2,
                   double* energy);

/* <S^2> of the current MPS, evaluated from the state: -N(N-4)/4 - 1/2
 * sum_ij Gamma^A_{ij;ji} with Gamma^A from one reverse pass (sadmrg_rdm).
 * The spin-adapted MPS is an exact spin eigenstate (section "Symmetry-adapted
 * DMRG"), so this returns S(S+1) to rounding; it checks the density matrix.
 * Errors: as sadmrg_rdm. */
int sadmrg_get_s2(sadmrg_ctx* ctx, double* s2);

/* ------------------------------------------------------------------------
 * MPS exchange.  Blob layout (little-endian, all fields int64 unless noted):
 *   magic 0x3154535053414453 ("SADSPST1"), L, N, twoS, irrep, centre i
 *   for bonds k = 0..L: nsec, then nsec x (N, twoS_sector, irrep, dim)
 *   left tensors  U[0..i-1]  as double: for each sector m of bond k+1 in
 *       order, a (dimX(m) x dim(m)) row-major matrix, rows in the left
 *       enlarged order (see below)
 *   right tensors V[i+2..L-1] as double: for each sector m of bond k, a
 *       (dim(m) x dimY(m)) row-major matrix, columns in the right enlarged order
 *   two-site object on sites (i, i+1) as double: for each sector m of bond
 *       i+1 present in both enlarged bases, a (dimX(m) x dimY(m)) matrix.
 * Sector labels (N, 2j, irrep) count the electrons LEFT of the bond; sectors
 * are sorted lexicographically.  Left enlarged order at bond k+1: pieces
 * (a, n) with a over bond-k sectors in order, then local state n in
 * (empty, single, double), keeping those with N_m = N_a + n_e, irrep
 * I_m = I_a x I(n), j_m in j_a (x) s_n.  Right enlarged order at bond k:
 * pieces (n, b), n outer, b over bond-(k+1) sectors, with N_b = N_m + n_e.
 * The two-site basis is [ |(a n1) j_M> (x) |(n2 b) j_M> ]^0 with the right
 * boundary's singlet-embedding spin S inside the right states.
 * ------------------------------------------------------------------------ */
int sadmrg_mps_import(sadmrg_ctx* ctx, const void* blob, size_t bytes);
int sadmrg_mps_export(sadmrg_ctx* ctx, void* blob, size_t* bytes); /* blob == NULL: size query */

/* ------------------------------------------------------------------------
 * Single-step hooks (test and benchmark access to one micro-iteration).
 * sadmrg_prepare_step builds the enlarged blocks for sites (i, i+1) where i
 * is the current centre; sadmrg_psi_layout reports nsec sectors, each as six
 * int64 (N, 2j, irrep, dimX, dimY, offset into the flat vector); and
 * sadmrg_sigma applies the effective Hamiltonian (section "The effective
 * Hamiltonian equation") to x[n] giving y[n].  x and y are device pointers
 * when on_device != 0, else host pointers.
 * ------------------------------------------------------------------------ */
int sadmrg_prepare_step(sadmrg_ctx* ctx);
/* Run n left-to-right micro-iterations (bond dimension D) from the current
 * centre, moving it right; *e_min receives their lowest energy. */
int sadmrg_advance(sadmrg_ctx* ctx, int D, int n, double* e_min);
/* Shapes of the prepared step's sigma tile tasks, five ints each (rows, K1,
 * K2, cols, flags of the triple-product record); size query when out == NULL. */
int sadmrg_debug_task_shapes(sadmrg_ctx* ctx, int* out, int64_t* n);
int sadmrg_psi_layout(sadmrg_ctx* ctx, int* nsec, int64_t* desc, int64_t* n);
int sadmrg_sigma(sadmrg_ctx* ctx, const double* x, double* y, int on_device);
/* sadmrg_sigma for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same FP64 sigma of the prepared step, y = H_eff x, with x[n] and y[n]
 * DEVICE pointers (may alias), enqueued on the context stream and finished
 * before return.  Every intermediate (the copies of x and y, the first GEMM
 * pass's workspace, the partial tiles of cut output tiles, and the launch
 * records) lives in one static device array of 32 MiB per device, allocated
 * when the library is loaded and held until the process ends; no device
 * memory is allocated or freed by this call.  The array keeps the last
 * call's contents; the output region is cleared on every call.  Calls are
 * serialised per device inside the process (a host lock held until the
 * stream is finished); calls that overlap on one device in any other way,
 * for instance work captured into a graph and replayed concurrently, race
 * on the array.  Results equal sadmrg_sigma's (same kernels, same order).
 * Errors: EINVAL (no prepared step, precision mode 1 or 2, or a step whose
 * intermediates exceed the array: the message gives the bytes needed),
 * EDEVICE. */
int sadmrg_sigma_noalloc(sadmrg_ctx* ctx, const double* x, double* y);

/* Diagonal of the effective Hamiltonian at the prepared step (same layout). */
int sadmrg_heff_diagonal(sadmrg_ctx* ctx, double* d, int on_device);

/* Initial vector of the prepared step's Davidson solve (same layout as
 * sadmrg_sigma): the current two-site object, moved to the prepared centre
 * by the decomposition of the previous step and the recoupling with the next
 * site tensor (section "The reduced two-site object", eqs. StoTT and TTtoS).
 * Read it before sadmrg_sigma with host vectors, which overwrites it.
 * out[n] is a device pointer when on_device != 0.  Errors: EINVAL. */
int sadmrg_debug_guess(sadmrg_ctx* ctx, double* out, int on_device);

/* Launch plan of the prepared step's FP64 sigma, out[6]: for the first and
 * then the accumulating GEMM pass, the number of tile pieces, of workgroups,
 * and of output tiles cut between workgroups (added by the ordered reduction).
 * Errors: EINVAL. */
int sadmrg_debug_plan_stats(sadmrg_ctx* ctx, int64_t* out);

/* Work counters of the prepared step's sigma: algorithmic flops (the sum
 * over block products c op(A) B op(C) of the two GEMMs' 2mnk, tile padding
 * excluded), bytes (every operator the products read, all its blocks, once,
 * plus the input and output vectors) and the number of block products. */
int sadmrg_sigma_counters(sadmrg_ctx* ctx, double* flops, double* bytes, int64_t* tasks);

/* Method-work counter.  The enlarged operator blocks the sigma products
 * multiply are dense (sector pair) blocks whose (sector, local state) piece
 * pairs are partly structurally zero.  With the counter on (on = 1), each
 * enlargement records its nonzero piece pairs and each prepared step counts
 * the flops of its sigma products with those zero pieces skipped (each
 * product in the cheaper of its two contraction orders); kept enlargements
 * are not used meanwhile (they carry no piece lists), which slows the sweep,
 * so turn it on for a counting sweep apart from timed ones.  Default off.
 * sadmrg_stats_method returns, since the last sadmrg_stats_reset, the method
 * flops and the performed flops (as sadmrg_stats) of the FP64 sigma calls on
 * counted steps, and the prepared step's method flops (-1 if not counted).
 * Errors: EINVAL. */
int sadmrg_set_method_counter(sadmrg_ctx* ctx, int on);
int sadmrg_stats_method(sadmrg_ctx* ctx, double* method_flops, double* performed_flops, double* step_method_flops);

/* Accumulated timings and counts since the last reset: seconds in sigma
 * kernels, number of sigma calls, seconds of whole micro-iterations, sigma
 * flops, and seconds in renormalisation/enlargement kernels. */
int sadmrg_stats(sadmrg_ctx* ctx, double* t_sigma, int64_t* n_sigma, double* t_micro, double* flops_sigma,
                 double* t_blocking);
int sadmrg_stats_reset(sadmrg_ctx* ctx);

/* Host wall seconds since the last reset of the parts of the micro-iterations
 * outside Davidson (section "Sweeping"), out[7]: enlargement of the two
 * blocks, sigma task lists, GEMM planning, effective-Hamiltonian diagonal,
 * initial guess, SVD and truncation, new site tensor and renormalisation.
 * Device work that these parts wait for is included.  Errors: EINVAL. */
int sadmrg_stats_phases(sadmrg_ctx* ctx, double* out);

/* Operator bytes touched by the sigma calls since the last reset (operator
 * stacks read + vector in/out, per call) and the largest enlarged-operator
 * footprint of one micro-iteration (both enlarged blocks). */
int sadmrg_stats_bytes(sadmrg_ctx* ctx, double* bytes_sigma, double* max_enlarged_bytes);
/* Sigma is evaluated by two grouped-GEMM launches (pass 1: T = X psi, pass 2:
 * sigma += T Y^T) plus an ordered reduction.  pass1[4] and pass2[4] receive,
 * since the last reset: kernel seconds (HIP events on the context stream
 * around each launch), algorithmic flops, algorithmic bytes (each GEMM
 * operand read once, each workspace/output block written once) and the number
 * of launches.  Either pointer may be NULL. */
int sadmrg_stats_passes(sadmrg_ctx* ctx, double* pass1, double* pass2);

/* FP32 sigma calls since the last reset: kernel seconds (conversions
 * included), count and algorithmic flops (same definition as FP64). */
int sadmrg_stats_mixed(sadmrg_ctx* ctx, double* t_sigma32, int64_t* n_sigma32, double* flops_sigma32);

/* Reference copy for HBM byte counters and bandwidth: allocates two device
 * arrays of n doubles, runs a plain streaming-copy kernel `reps` times on the
 * context stream (8n bytes read + 8n bytes written per launch) and returns
 * the mean kernel seconds per launch.  Frees both arrays.  Errors: EINVAL
 * (n or reps not positive), ENOMEM, EDEVICE. */
int sadmrg_debug_copy_probe(sadmrg_ctx* ctx, int64_t n, int reps, double* seconds);

/* Reference GEMM for HBM byte counters: nprod independent products
 * c_q = a_q b_q (64 x K times K x 64, every operand its own array, so each
 * is read once and each result written once) through the sigma pass-1
 * kernel (one 64 x 64 tile per workgroup), `reps` launches; *seconds gets
 * the mean kernel time per launch, *bytes the exact traffic per launch
 * (8 (2 * 64 K + 64 * 64) nprod).  Allocates and frees its arrays.  Errors:
 * EINVAL (sizes), ENOMEM, EDEVICE. */
int sadmrg_debug_gemm_probe(sadmrg_ctx* ctx, int nprod, int K, int reps, double* seconds, double* bytes);

/* Description of the last failure (static until the next call on ctx). */
const char* sadmrg_last_error(const sadmrg_ctx* ctx);

/* Debug/test access to the library's SU(2) recoupling coefficients (spins
 * doubled).  which = 0: coupled product of operators on two subsystems,
 * args[9] = (j1, j2, J, k1, k2, K, j1', j2', J') through a Wigner 9j symbol;
 * which = 1: same-space product, args[6] = (j, j'', j', k1, k2, K) through a
 * 6j symbol; which = 2: 6j symbol {a b c; d e f}, args[6].  Returns the value
 * in *out. */
int sadmrg_debug_coupling(int which, const int* args, double* out);

#ifdef __cplusplus
}
#endif
#endif /* SADMRG_H */
