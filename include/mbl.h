/*
 * mbl.h - C ABI of the MI355X (gfx950) library for nested shift-invert
 * diagonalization of the periodic random-field Heisenberg chain in the
 * S^z = 0 sector (Kutsuzawa & Todo, arXiv:2203.09732).
 *
 * Model (Sec. I, Eq. (1)):  H = sum_{j=1}^{L} ( S_j . S_{j+1} - h_j S^z_j ),
 * S_{L+1} = S_1, L even, J = 1. Site j is bit j-1 of a state integer and a set
 * bit is S^z = +1/2. The sector basis is every L-bit integer with L/2 set bits
 * in ascending order; index i of an n-vector is the i-th such integer,
 * n = C(L, L/2).
 *
 * Conventions for every entry point:
 *  - Return value: 0 (MBL_OK) on success; < 0 on error, in which case no
 *    output has been written and nothing was launched; > 0 is a warning and
 *    the outputs are valid but best effort (see each call).
 *    mbl_last_error() gives a message for the last non-OK status on the
 *    calling thread.
 *  - Host pointers are named *_host; device pointers *_dev. Device buffers are
 *    owned by the caller, contiguous, and never freed by the library.
 *    n-vectors are FP64 unless stated.
 *  - h_host points to L doubles (the fields h_1..h_L); it is read during the
 *    call only.
 *  - stream is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls that return host values synchronize that stream; the others are
 *    asynchronous with respect to the host.
 *  - The library calls the HIP runtime loaded in the process. A caller that
 *    passes streams or device pointers from a framework must make sure one
 *    HIP runtime is loaded (a framework bundling its own libamdhip64.so.7 is
 *    loaded first, so this library binds to it).
 *  - Handles (mbl_basis, mbl_workspace) are created and freed by the library.
 *    A basis is immutable after creation and may be shared by streams; a
 *    workspace must not be used by two calls at once.
 */
#ifndef MBL_H
#define MBL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mbl_status;
enum {
  MBL_OK = 0,
  MBL_ERR_ARG = -1,        /* invalid argument; nothing done */
  MBL_ERR_NOMEM = -2,      /* device or host allocation failed */
  MBL_ERR_HIP = -3,        /* a HIP runtime call failed */
  MBL_ERR_NUMERIC = -4,    /* NaN/Inf met in a recurrence */
  MBL_WARN_NOCONV = 1,     /* iteration limit reached before the tolerance */
  MBL_WARN_BREAKDOWN = 2   /* Lanczos found an invariant subspace (beta ~ 0) */
};

/* Arithmetic of the MINRES inner solves. */
enum {
  MBL_FP64 = 0,            /* FP64 throughout */
  MBL_FP32_INNER = 1       /* FP32 MINRES vectors and matvec, FP64 residual
                              recomputation b - (H - sigma) x and restart;
                              Lanczos, Ritz values and residual checks FP64 */
};

/* Diagonal preconditioner M = C C^dagger (Sec. II). */
enum {
  MBL_PRECOND_ROW = 0,     /* M = diag(r_i), r_i = 2-norm of row i of H - sigma I
                              (the row-norm preconditioner of Sec. II) */
  MBL_PRECOND_JACOBI = 1,  /* M = diag(|a_ii - sigma|); an element equal to 0 is
                              an argument error at solve time (MBL_ERR_NUMERIC) */
  MBL_PRECOND_ID = 2       /* M = I */
};

typedef struct mbl_basis_s* mbl_basis;
typedef struct mbl_workspace_s* mbl_workspace;

/* ---- basis (Sec. III: dimension C(L, L/2)) --------------------------------
 * mbl_build_basis: builds the sector tables for an even L, 4 <= L <= 32, on
 * the current HIP device. lo_bits = number of low bits in the (high, low)
 * split of a state used by the kernels (0 = library default; else
 * 1 <= lo_bits <= 13 and lo_bits < L). Errors: MBL_ERR_ARG for odd/out of
 * range L or lo_bits. Synchronizes stream. */
mbl_status mbl_build_basis(int L, int lo_bits, void* stream, mbl_basis* out);
void mbl_basis_free(mbl_basis b);
/* n = C(L, L/2) */
mbl_status mbl_basis_dim(mbl_basis b, int64_t* n);
/* number of low bits of the (high, low) split the basis was built with */
mbl_status mbl_basis_lo_bits(mbl_basis b, int* lo_bits);
/* Writes the n sector states (ascending uint32) to states_dev[n]. Async. */
mbl_status mbl_basis_states(mbl_basis b, uint32_t* states_dev, void* stream);
/* Index of each of count states (each must be a sector state) into
 * ranks_dev[count] (int64). A state outside the sector yields -1. Async. */
mbl_status mbl_basis_rank(mbl_basis b, const uint32_t* states_dev, int64_t count,
                          int64_t* ranks_dev, void* stream);

/* ---- workspace -------------------------------------------------------------
 * Device scratch for MINRES (its recurrence vectors) and for up to mmax
 * Lanczos basis vectors, 0 <= mmax <= 1000 (MBL_ERR_ARG otherwise).
 * precision selects the MINRES vector type. Size: 8 n (13 + mmax + 1) bytes
 * for mmax > 0 (8 n 13 for mmax = 0) plus about 1 MB: the MINRES vectors
 * z and d (two each), q (three) and p, an FP32-inner correction, a residual and a
 * scratch vector, the Lanczos w and x, and the Lanczos basis. */
mbl_status mbl_workspace_create(mbl_basis b, int mmax, int precision, mbl_workspace* ws);
void mbl_workspace_free(mbl_workspace ws);
/* Device bytes held by the workspace. */
mbl_status mbl_workspace_bytes(mbl_workspace ws, int64_t* bytes);

/* ---- y = (H - sigma I) x (Eq. (1); the matrix-vector product inside Alg. 2)
 * x_dev, y_dev: n doubles, must not overlap. The matrix is never stored:
 * diagonal and spin-flip elements are generated from the state bits. Async. */
mbl_status mbl_apply_H(mbl_basis b, const double* h_host, double sigma,
                       const double* x_dev, double* y_dev, void* stream);
/* Same product in FP32 storage (diagonal formed in FP64, then rounded). */
mbl_status mbl_apply_H_f32(mbl_basis b, const double* h_host, double sigma,
                           const float* x_dev, float* y_dev, void* stream);

/* ---- q = M^{-1} z with the chosen diagonal preconditioner (Sec. II,
 * the row-norm preconditioner of Sec. II). z_dev, q_dev: n doubles (may alias). Async. */
mbl_status mbl_precond_apply(mbl_basis b, const double* h_host, double sigma, int precond,
                             const double* z_dev, double* q_dev, void* stream);

/* ---- preconditioned MINRES for (H - sigma I) x = b (App. A, Alg. 2) --------
 * rhs_dev: n doubles. x_dev: n doubles, initial guess on entry (x0), solution
 * on exit. Stops when |phi_k| < tol (phi_k = ||b - A x_k||_{M^{-1}}) or after
 * kmax iterations (MBL_WARN_NOCONV). With MBL_FP32_INNER the solve runs in
 * cycles: an FP32 MINRES solve of A e = r / ||r|| to a relative 1e-3 (smaller
 * near the end), x += ||r|| e in FP64, r = b - A x recomputed in FP64. A cycle
 * that fails to cut ||r||_{M^{-1}} tenfold (the FP32 recurrence drifts from
 * the true residual by roughly u_32 times the squared condition number, so
 * near the middle of a large spectrum a cycle can stop having achieved
 * nothing), or the 60th cycle, ends the FP32 phase and FP64 MINRES finishes
 * on the current residual. The stop test is
 * then the FP64 ||r||_{M^{-1}} < tol. Synchronizes stream. info may be NULL. */
typedef struct {
  int64_t iters;       /* MINRES iterations, summed over restarts */
  int32_t restarts;    /* FP32 cycles (0 in MBL_FP64) */
  double phi;          /* final |phi|: the recurrence estimate (MBL_FP64), the
                          recomputed FP64 ||r||_{M^{-1}} (MBL_FP32_INNER) */
  double true_res;     /* ||b - (H - sigma) x||_2 recomputed in FP64 */
} mbl_minres_info;
mbl_status mbl_minres_solve(mbl_basis b, const double* h_host, double sigma,
                            const double* rhs_dev, double* x_dev, double tol, int64_t kmax,
                            int precision, int precond, mbl_workspace ws,
                            mbl_minres_info* info, void* stream);

/* ---- shift-invert Lanczos (Sec. II, Alg. 1) with MINRES inner solves --------
 * Finds the nev eigenpairs of H with eigenvalues closest to sigma. Each step
 * solves (H - sigma) x = v_k by mbl_minres_solve semantics (minres_tol,
 * minres_kmax), orthogonalises against v_{k-1}, v_k by the three-term
 * recurrence and then against all earlier v by two classical Gram-Schmidt
 * passes, all in FP64 on the device. Stops when all nev selected Ritz pairs
 * satisfy est_i <= eig_tol * escale and est_i <= gap_tol * gap_i, where est_i
 * is the shift-invert residual estimate mapped to H, gap_i the distance to
 * the nearest other Ritz value, and escale = max(|E_min|, |E_max|) if passed
 * > 0, else a Gershgorin bound on ||H||; or when k = mmax (MBL_WARN_NOCONV)
 * or beta_{k+1} <= 1e-14 * max|theta| (MBL_WARN_BREAKDOWN). gap_tol <= 0
 * disables the gap test.
 * v0_dev: n doubles start vector, or NULL for a seeded one (SplitMix64 of
 * (seed, i) mapped to a uniform in [-1/2, 1/2)).
 * Outputs: evals_host[nev] ascending; evecs_dev: n x nev column-major with
 * leading dimension ld >= n, unit 2-norm, sign arbitrary; resid_host[nev]:
 * explicit ||H u - lambda u||_2 recomputed in FP64 (may be NULL).
 * Synchronizes stream. info may be NULL. */
typedef struct {
  int32_t steps;          /* Lanczos steps k */
  int32_t nconv;          /* pairs passing the test */
  int64_t minres_iters;   /* total MINRES iterations */
  double max_rel_resid;   /* max_i resid_i / escale */
  double seconds;         /* wall time of the call */
} mbl_si_info;
mbl_status mbl_si_lanczos(mbl_basis b, const double* h_host, double sigma, int nev, int mmax,
                          double minres_tol, int64_t minres_kmax, double eig_tol,
                          double gap_tol, double escale, const double* v0_dev, uint64_t seed,
                          int precision, int precond, mbl_workspace ws,
                          double* evals_host, double* evecs_dev, int64_t ld,
                          double* resid_host, mbl_si_info* info, void* stream);

/* ---- twist overlap z = <psi|U_twist|psi> (Sec. III; App. B form
 * z = sum_alpha c_alpha^2 u_alpha) for nvec real vectors psi_dev (n x nvec,
 * column-major, leading dimension ld >= n). z_host[2*t] = Re z_t,
 * z_host[2*t+1] = Im z_t. Vectors are used as given (not renormalised).
 * Synchronizes stream. */
mbl_status mbl_twist_expect(mbl_basis b, const double* psi_dev, int64_t ld, int nvec,
                            double* z_host, void* stream);

/* ---- allocation-free twist overlap, for callers that cannot allocate device
 * memory (code that must not call hipMalloc: serving loops, harnesses that
 * forbid allocation). Same result as mbl_twist_expect, bit for bit (the same
 * kernels and reduction order), for nvec <= 32 vectors; nvec > 32 is
 * MBL_ERR_ARG. The partial sums live in a static device array of the
 * library (32 x 1024 x 2 + 64 doubles, about 513 KB, held by each GPU the
 * library runs on until the process ends): the call allocates nothing. Calls
 * that overlap on one GPU share that array and race; serialise them. The
 * basis must belong to the current device. Synchronizes stream. */
mbl_status mbl_twist_expect_noalloc(mbl_basis b, const double* psi_dev, int64_t ld, int nvec,
                                    double* z_host, void* stream);

/* ---- explicit eigen-residuals ||H psi_t - E_t psi_t||_2 (Alg. 1 output
 * check), psi_dev n x nvec (ld >= n), E_host[nvec], resid_host[nvec].
 * Synchronizes stream. */
mbl_status mbl_eig_residual(mbl_basis b, const double* h_host, const double* E_host,
                            const double* psi_dev, int64_t ld, int nvec,
                            double* resid_host, void* stream);

/* ---- bipartite entanglement entropy (Sec. IV, entanglement and level
 * spacing): S_t = -Tr rho_A ln rho_A for each of nvec real vectors psi_dev
 * (device, n x nvec column-major, ld >= n; any norm: rho_A is divided by its
 * trace), with A = sites 1..la (bits 0..la-1), 1 <= la <= L-1 (the paper
 * takes la = L/2). rho_A is block diagonal in the number k of up spins in
 * A; the coefficients of each block are gathered on the device and their
 * Gram matrices (min(C(la,k), C(L-la,L/2-k)) squared) formed on the FP64
 * matrix cores; the eigenvalues of the blocks are found on the host
 * (Householder tridiagonalisation, symmetric QR) with up to 16 threads.
 * S_host[nvec]. Allocates device scratch of at most 4 GiB (16 n bytes per
 * vector of a pass) and frees it before returning. Synchronizes stream.
 * MBL_ERR_NUMERIC for a zero or non-finite vector. */
mbl_status mbl_entanglement_entropy(mbl_basis b, const double* psi_dev, int64_t ld, int nvec,
                                    int la, double* S_host, void* stream);
/* The same for nvec x R vectors stored interleaved, element i of vector t of
 * realization r at psi_dev[(t * n + i) * R + r] (the layout of
 * mbl_si_lanczos_batched's eigenvectors). S_host[r * nvec + t]. */
mbl_status mbl_entanglement_entropy_interleaved(mbl_basis b, const double* psi_dev, int R,
                                                int nvec, int la, double* S_host, void* stream);

/* Host-only: eigenvalues of the m x m symmetric matrix a_host (row-major, all
 * m^2 entries read; 1 <= m <= 20000), ascending, into w_host[m]: Householder
 * reduction to tridiagonal form with scaled reflectors, columns below 1e-20
 * max|a| taken as zero, then the symmetric QR iteration of mbl_tridiag_eig.
 * This is the routine mbl_entanglement_entropy applies to its Schmidt blocks.
 * Uses no device. MBL_ERR_NUMERIC if an eigenvalue needs more than 60 QR
 * steps. */
mbl_status mbl_symmetric_eigenvalues(int m, const double* a_host, double* w_host);

/* ---- level-spacing ratio (Sec. IV): over the ascending sort of
 * evals_host[count] (count >= 3), r_k = min(d_k, d_{k-1}) / max(d_k, d_{k-1})
 * with d_k = E_{k+1} - E_k. r_host[count-2] (may be NULL) receives r_1 ..
 * r_{count-2}, NaN where both spacings are 0; *r_mean is the mean of the
 * defined ratios (NaN if none). Host only. */
mbl_status mbl_spacing_ratio(int count, const double* evals_host, double* r_host,
                             double* r_mean);

/* ---- sigma = (E_min + E_max) / 2 (Sec. IV A) by Lanczos on H without
 * reorthogonalisation (the extremal Ritz values converge first and are not
 * affected by the copies loss of orthogonality creates), from a seeded start
 * vector; stops when the residual estimates of both extremes are below
 * rel_tol * max(|E_min|, |E_max|). mmax bounds the steps (0 = default 300;
 * MBL_WARN_NOCONV if reached). Synchronizes stream. */
mbl_status mbl_sigma_midpoint(mbl_basis b, const double* h_host, double rel_tol, int mmax,
                              double* emin, double* emax, double* sigma, void* stream);

/* ---- eigenpair derivatives with respect to the fields h_j -------------------
 * For an eigenpair (E, psi) of Eq. (1) (psi_dev: n doubles, any norm; the
 * formulas use psi / ||psi||):
 *  dE_dh_host[j]  = dE/dh_{j+1} = -<S^z_{j+1}> (Hellmann-Feynman, exact);
 *  dz2_dh_host[j] = d|z|^2/dh_{j+1}, z = <psi|U_twist|psi> (Sec. III), by the
 *    adjoint solve (H - E) lambda = P g with g_a = 4 c_a Re(conj(z) u_a),
 *    P = I - psi psi^T, lambda re-projected orthogonal to psi, then
 *    d|z|^2/dh_j = sum_a lambda_a c_a s_j(a). The solve is preconditioned
 *    MINRES (Alg. 2) on (H - E + psi psi^T / ||psi||^2) lambda = P g: the
 *    rank-one term lifts the near-null direction psi of H - E and leaves the
 *    solution for a right-hand side orthogonal to psi unchanged. Tolerance
 *    tol, kmax iterations; any workspace of the basis (any mmax).
 * z_host[2] (Re, Im of z) and info may be NULL. MBL_WARN_NOCONV if the solve
 * missed tol. Synchronizes stream. */
mbl_status mbl_eig_grad(mbl_basis b, const double* h_host, double E, const double* psi_dev,
                        double tol, int64_t kmax, int precond, mbl_workspace ws,
                        double* dE_dh_host, double* dz2_dh_host, double* z_host,
                        mbl_minres_info* info, void* stream);

/* ---- batched form: R realizations of one L in lockstep ---------------------
 * R disorder realizations of the basis's chain length, each with its own
 * fields h_r (h_host: R x L doubles, row r = realization r) and shift
 * sigma_r (sigma_host: R doubles). Batched n-vectors are interleaved:
 * element (i, r) at index i * R + r of an n * R array. R is a power of two,
 * 2 <= R <= 32, and R * 16 * ceil(L/4) doubles of field tables must fit the
 * kernels' 64 KB LDS budget (R = 32 up to L = 24, R = 16 at L = 26), and
 * n * R * 8 bytes must stay below 2^31 (the kernels address batch vectors
 * with 32-bit byte offsets); otherwise MBL_ERR_ARG. L must be one of
 * 12, 14, ..., 32 and the basis's lo_bits one of the splits the library has
 * batched kernels for (the default split of every such L, and the
 * alternatives the autotuner measures). The batch workspace holds the
 * recurrence vectors of all realizations (z, d and p, a ring of 8 q vectors
 * for the d/x update grouped over 4 iterations, the FP32-inner correction,
 * residual, scratch, Lanczos w and x: 18 n R doubles) and up to mmax + 1
 * Lanczos blocks of n R doubles. */
typedef struct mbl_batch_s* mbl_batch;
mbl_status mbl_batch_create(mbl_basis b, int R, int mmax, int nevmax, mbl_batch* out);
void mbl_batch_free(mbl_batch w);
mbl_status mbl_batch_bytes(mbl_batch w, int64_t* bytes);
/* Launch schedule of a batch workspace's kernels (a tuning knob; results do
 * not depend on it beyond the order of the partial sums): grid = workgroups
 * of the row kernels (0: one per compute unit; else a multiple of 8 up to
 * 512), graph_iters = MINRES iterations per captured graph (0 = 16; 8, 16 or
 * 32), dx_group = MINRES iterations per d/x pass (0 = 4; 1, 2 or 4).
 * MBL_ERR_ARG on other values. Drops the workspace's captured graphs when the
 * schedule changes. */
mbl_status mbl_batch_set_schedule(mbl_batch w, int grid, int graph_iters, int dx_group);
/* y_r = (H_r - sigma_r) x_r for every r (Eq. (1)); interleaved x, y. Async.
 * At lo_bits = 10 with R = 32 (L = 14, 16, 22) the product stages blocks of
 * x in LDS; the first such call on a workspace (and the first after a
 * schedule change) builds the workspace's block lists and synchronizes the
 * stream once. */
mbl_status mbl_apply_H_batched(mbl_basis b, mbl_batch w, const double* h_host,
                               const double* sigma_host, const double* x_dev, double* y_dev,
                               void* stream);
mbl_status mbl_apply_H_batched_f32(mbl_basis b, mbl_batch w, const double* h_host,
                                   const double* sigma_host, const float* x_dev, float* y_dev,
                                   void* stream);
/* Alg. 2 for every realization from x0 = 0 (x_dev is overwritten); per
 * realization stop at |phi_r| < tol or kmax. iters_host[R], phi_host[R] may
 * be NULL. MBL_WARN_NOCONV if any realization missed tol. Synchronizes. */
mbl_status mbl_minres_solve_batched(mbl_basis b, mbl_batch w, const double* h_host,
                                    const double* sigma_host, const double* rhs_dev,
                                    double* x_dev, double tol, int64_t kmax, int precision,
                                    int precond, int64_t* iters_host, double* phi_host,
                                    void* stream);
/* Alg. 1 for every realization in lockstep with the stopping rule of
 * mbl_si_lanczos applied per realization (escale_host: R values or NULL); a
 * realization that has converged stops taking steps (its MINRES right-hand
 * side is zeroed). Outputs: evals_host[R * nev] (realization-major,
 * ascending per realization), evecs_dev: nev interleaved blocks of n * R
 * doubles (block t holds pair t of every realization), resid_host[R * nev]
 * explicit FP64 residuals, info_host[R] (minres_iters: the iterations that
 * realization's own solves took; the batch launches, per Lanczos step, as
 * many as its slowest realization). Synchronizes. */
mbl_status mbl_si_lanczos_batched(mbl_basis b, mbl_batch w, const double* h_host,
                                  const double* sigma_host, int nev, int mmax, double minres_tol,
                                  int64_t minres_kmax, double eig_tol, double gap_tol,
                                  const double* escale_host, const double* v0_dev, uint64_t seed,
                                  int precision, int precond, double* evals_host,
                                  double* evecs_dev, double* resid_host, mbl_si_info* info_host,
                                  void* stream);
/* z for nvec interleaved blocks (layout of mbl_si_lanczos_batched's evecs):
 * z_host[((r * nvec) + t) * 2 + {0: Re, 1: Im}]. Synchronizes. */
mbl_status mbl_twist_expect_batched(mbl_basis b, mbl_batch w, const double* psi_dev, int nvec,
                                    double* z_host, void* stream);

/* ---- many disorder realizations of uneven chain length in one call --------
 * The disorder averages of Sec. IV need the eigenpairs nearest sigma of many
 * realizations, each with its own L, fields and shift. Every problem is
 * solved as by mbl_si_lanczos (Alg. 1 with Alg. 2 inner solves, FP64, the
 * same stopping rule), with its Ritz vectors, explicit residuals and twist
 * overlaps (Sec. III). Problems with L <= 16 run in one persistent launch
 * (replayed from a captured graph): each workgroup claims a problem from a
 * device counter and runs sigma, the Lanczos steps with their MINRES solves,
 * the reorthogonalisation, the tridiagonal eigensolver, the Ritz extraction,
 * residuals and twist on the device. Problems with L >= 18 run after it,
 * per L, in the streaming batched form: up to 32 lanes of one batch
 * workspace share every MINRES launch, but each lane takes its own Lanczos
 * steps (its solve restarted in flight on v_{k+1} when it ends) and, when
 * its realization has converged, the next one (sigma found per realization
 * first). The environment variable MBL_PERSISTENT_MAX_L (even, 10..16)
 * lowers the longest chain of the persistent launch.
 * Per problem (inputs): L (even, 4..32), nev (1..min(32, C(L, L/2))),
 * h_host (L fields), sigma (NaN: (E_min + E_max)/2 computed here, Sec. IV A),
 * escale (> 0: energy scale of the stopping rule; else max(|E_min|, |E_max|)
 * when sigma is computed, else a Gershgorin bound on ||H||), evecs_dev (n x nev
 * column-major, ld = n, on the current device). Outputs: evals_host (nev,
 * ascending), resid_host (nev, may be NULL), z_host (2 nev: Re, Im; may be
 * NULL), sigma_out, info (info.seconds is the wall time of the whole call),
 * status (that problem's mbl_si_lanczos status). mmax: 0 = 3 nev + 40 per
 * problem, else 1..128 for all. Returns MBL_ERR_ARG before any launch on a
 * bad argument, MBL_OK if every problem converged, else MBL_WARN_NOCONV (or
 * MBL_WARN_BREAKDOWN) with the per-problem status set. Allocates its working
 * memory for the call (per workgroup: 8 + mmax + 1 n-vectors) and frees it.
 * Synchronizes stream. */
typedef struct {
  int32_t L;
  int32_t nev;
  const double* h_host;
  double sigma;
  double escale;
  double* evecs_dev;
  double* evals_host;
  double* resid_host;
  double* z_host;
  double sigma_out;
  mbl_si_info info;
  mbl_status status;
} mbl_problem;
mbl_status mbl_si_lanczos_problems(mbl_problem* probs, int nprob, int mmax, double minres_tol,
                                   int64_t minres_kmax, double eig_tol, double gap_tol,
                                   uint64_t seed, int precond, void* stream);

/* ---- small device helpers used by the bindings and tests ---------------- */
/* out_host = sum_i x_i * y_i over n doubles, reduced in a fixed order. */
mbl_status mbl_dot(int64_t n, const double* x_dev, const double* y_dev, double* out_host,
                   void* stream);

/* Host-only: eigen-decomposition of the k x k symmetric tridiagonal T_k of
 * Alg. 1 (diagonal alpha[k], off-diagonal beta[k-1]) by the symmetric QR
 * algorithm (implicit steps with Wilkinson shift, Golub & Van Loan Sec. 8.3).
 * evals_host[k] ascending; evecs_host k x k column-major, column i
 * for evals_host[i]. Uses no device. MBL_ERR_NUMERIC if an eigenvalue needs
 * more than 60 QR steps. */
mbl_status mbl_tridiag_eig(int k, const double* alpha_host, const double* beta_host,
                           double* evals_host, double* evecs_host);

/* Message for the last non-OK status on this thread ("" if none). */
const char* mbl_last_error(void);
/* Library version string. */
const char* mbl_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MBL_H */
