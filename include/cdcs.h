/*
 * cdcs.h -- C ABI of the MI355X (gfx950) HSDE-ADMM for chordally sparse SDPs.
 *
 * The solver computes the ADMM iteration of Zheng, Fantuzzi,
 * Papachristodoulou, Goulart & Wynn, "Fast ADMM for homogeneous self-dual
 * embedding of sparse SDPs": the primal/dual pair of Section 3 (eqs.
 * PrimalSDP / DualSDP), decomposed over the maximal cliques of a chordal
 * pattern (Theorems 1-2, eqs. DecomposedPriaml / DecomposedDual), embedded
 * as in Section 3.2 (eq. HomogeneousEmbedding) and iterated with steps
 * (Step1)-(Step3) of Section 4.1, where step 1 uses the block eliminations
 * and the matrix inversion lemma of Sections 4.2-4.3.
 *
 * Conventions (all entry points):
 *  - Indices are 0-based int32.  Symmetric matrices (C and every A_i) are
 *    given as lower-triangular COO (row >= col); an off-diagonal entry (i,j)
 *    stands for both X_ij and X_ji.  Duplicate entries are summed.
 *  - Cliques: p vertex lists in CSR form (clique_ptr[p+1], clique_vtx), each
 *    list strictly increasing (the natural order of Section 2.1) and of at
 *    most 1024 vertices (CDCS_E_CLIQUES otherwise).  Every vertex must lie in
 *    some clique and every data entry inside some C_k x C_k (the chordal
 *    pattern E').  The m x m matrix of step 1 is factorised densely when it
 *    is at least 20 % full and m <= 2048 (or m <= 64), sparsely otherwise
 *    (any m).  The optional clique_parent array
 *    (p entries, -1 = root) is checked for the running-intersection
 *    property.  Chordal extension and clique-tree construction are done by
 *    the caller on the host.
 *  - Coordinates.  Vectors over the pattern ("entry space") hold svec of a
 *    symmetric matrix over the lower entries of E' (off-diagonals scaled by
 *    sqrt 2) in canonical order: sorted by column, then row.  Clique blocks
 *    ("slot space": s, z, v) are stored clique after clique in the given
 *    clique order, each as the packed lower triangle in column-major local
 *    order, off-diagonals scaled by sqrt 2.  This is an isometry of the
 *    paper's vec coordinates on symmetric matrices.
 *  - State u = (x, s, y, v, tau) and v~ = (h, z, r, w, kappa) of eq.
 *    (ADMMForm) are flattened in that block order; each has length
 *    nE + 2 ns + m + 1.
 *  - Return values: 0 = OK, negative = error (CDCS_E_*), with a message
 *    from cdcs_last_error() (thread-local).  Nothing throws across the ABI.
 *    Solver outcomes (infeasible, iteration limit) are reported in
 *    cdcs_info.status, not as errors.
 *  - Ownership: inputs are copied during setup; the caller may free them on
 *    return.  The handle owns all device memory until cdcs_destroy.  Output
 *    buffers are caller-allocated.  A handle must not be used from two
 *    threads at once.  All device work runs on the stream given at setup
 *    (NULL = the default stream); host-pointer outputs synchronise it.
 */
#ifndef CDCS_H
#define CDCS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CDCS_ABI_VERSION 6

/* outcomes (cdcs_info.status) */
enum {
  CDCS_RUNNING = 0,
  CDCS_SOLVED = 1,
  CDCS_PRIMAL_INFEASIBLE = 2,
  CDCS_DUAL_INFEASIBLE = 3,
  CDCS_MAX_ITER = 4
};

/* cdcs_settings.method */
enum {
  CDCS_METHOD_SELF_DUAL = 0, /* the ADMM of eqs. Step1-Step3 on the homogeneous self-dual embedding */
  CDCS_METHOD_PRIMAL = 1,    /* primal-only ADMM of the authors' earlier work (Section 5, CDCS-primal) */
  CDCS_METHOD_DUAL = 2       /* dual-only ADMM of the authors' earlier work (Section 5, CDCS-dual) */
};

/* errors (negative return values) */
enum {
  CDCS_OK = 0,
  CDCS_E_ARG = -1,        /* null pointer, size out of range, bad setting */
  CDCS_E_PATTERN = -2,    /* a C or A_i entry outside the union of C_k x C_k */
  CDCS_E_CLIQUES = -3,    /* unsorted/out-of-range clique, uncovered vertex, tree violates running intersection */
  CDCS_E_NONFINITE = -4,  /* NaN or Inf in the data */
  CDCS_E_FACTOR = -5,     /* the m x m factorisation failed */
  CDCS_E_DEVICE = -6,     /* a HIP call failed */
  CDCS_E_NOMEM = -7,      /* device or host allocation failed */
  CDCS_E_STATE = -8       /* call not valid in the handle's current state */
};

typedef struct cdcs_handle cdcs_handle;

/* One SDP instance: min <C,X> s.t. <A_i,X> = b_i, X PSD (eq. PrimalSDP),
 * with the cliques C_1..C_p of a chordal extension of its pattern. */
typedef struct {
  int32_t n;                 /* order of X */
  int32_t m;                 /* number of equality constraints */
  int64_t c_nnz;             /* entries of C (lower COO) */
  const int32_t* c_row;
  const int32_t* c_col;
  const double* c_val;
  int64_t a_nnz;             /* entries of all A_i (lower COO + constraint id) */
  const int32_t* a_con;      /* constraint index i in [0, m) */
  const int32_t* a_row;
  const int32_t* a_col;
  const double* a_val;
  const double* b;           /* m values */
  int32_t p;                 /* number of cliques */
  const int32_t* clique_ptr; /* p + 1 offsets into clique_vtx */
  const int32_t* clique_vtx; /* vertex lists, strictly increasing per clique */
  const int32_t* clique_parent; /* p parents (-1 = root) or NULL */
} cdcs_problem;

typedef struct {
  double eps_tol;      /* termination tolerance (Section 5: 1e-4) */
  int32_t max_iter;    /* iteration limit (Section 5: 2000) */
  int32_t check_every; /* cdcs_solve reads the status words back every this many iterations */
  int32_t timing;      /* 1 = time each kernel phase with HIP events (cdcs_get_phase_times) */
  int32_t use_graph;   /* 1 = replay the iteration from a captured HIP graph */
  int32_t eig_fp32;    /* 1 = eigen-decompose cliques of up to 64 vertices in FP32 (Jacobi in
                          FP32; gather, Y and the update of s, z, v stay FP64); larger cliques
                          always FP64.  The iterates then differ from the FP64 method by ~1e-7
                          relative per conic step. */
  int32_t autotune;    /* Jacobi tile shape (threads per clique) of every clique-size bucket:
                          0 = the default shape; 1 = at setup, time both candidate shapes on
                          synthetic blocks of the instance's clique orders and keep the
                          faster; 2 = the other candidate without timing (for comparisons).
                          cdcs_get_tuning reports the choice. */
  double alpha;        /* relaxation of steps 2-3, in (0, 2): they take
                          alpha u_hat + (1 - alpha) u in place of u_hat, the
                          over-relaxed form of the ADMM of O'Donoghue et al.
                          2016 that Section 4.1 applies (same fixed points).
                          1 = eqs. Step2-Step3 exactly (the default).  Other
                          values add, per iteration, one pass of A over x, of
                          A^T over y and of H^T over v of the previous iterate
                          inside the existing kernels, and 4 vectors (3 nE,
                          1 m) of device memory; otherwise CDCS_E_ARG. */
  int32_t eig_warm;    /* 1 = start the Jacobi eigen-decomposition of every clique of up to 64
                          vertices from its eigenvectors of the previous iteration (Y is
                          rotated to V^T Y V, nearly diagonal once the iterates settle, and
                          the sweeps continue from there); the projection is the same up to
                          rounding (it is unique).  Cold starts: the first iteration, the
                          first after cdcs_set_state, and every 64th.  Costs sum_k K_k^2
                          values of device memory.  A resumed run then matches an
                          uninterrupted one to rounding, not bit for bit.  0 = off. */
  int32_t method;      /* CDCS_METHOD_SELF_DUAL (default), or one of the two methods Section 5
                          compares with: the primal-only and dual-only ADMM of the authors'
                          earlier chordal-decomposition work (CDCS-primal, CDCS-dual), the
                          textbook ADMM on the consensus constraint s = H x (primal form,
                          eq. DecomposedPriaml) or v = z (dual form, eq. DecomposedDual) with
                          penalty rho.  Their step 1 solves with the m x m matrix A D^-1 A^T
                          (factorised at setup, D = H^T H; CDCS_E_FACTOR if the constraints are
                          linearly dependent on the pattern), their step 2 is the same clique
                          projection.  They stop when eps_p = ||s - Hx|| / max(||s||, ||Hx||)
                          (primal; dual: ||v - z|| / max(||v||, ||z||)) and eps_d =
                          rho ||s+ - s|| / ||lam|| (dual: z) are both within eps_tol; they
                          detect no infeasibility (status SOLVED or MAX_ITER only) and take
                          alpha = 1, eig_warm = 0 and no adjoint (CDCS_E_ARG otherwise). */
  double rho;          /* penalty of the primal-only / dual-only methods (> 0; default 1) */
  int32_t jacobi_max;  /* largest clique order the Jacobi kernels take: 16, 32 or 64; 0 = 32, or
                          64 when eig_fp32 or eig_warm is on;
                          larger cliques take the tridiagonal path (reduction in LDS up to 136
                          vertices, then bisection, inverse iteration and back-transformation).
                          The projection is the same (it is unique); only the route and its cost
                          change.  eig_fp32 and eig_warm apply to the Jacobi cliques only. */
  int32_t band_min;    /* smallest clique order whose eigendecomposition starts with the two-stage
                          reduction (dense to a band of 8 sub-diagonals by panel QR, then band
                          to tridiagonal by bulge chasing in LDS); smaller cliques above the
                          Jacobi sizes take the one-stage blocked reduction (its last 136
                          columns in LDS).  0 = automatic: 137 (every clique the LDS
                          reduction cannot hold whole) when the largest clique has at least 320
                          vertices, otherwise none (a lone clique of a few hundred vertices is
                          reduced faster by the one-stage path); values above 1024 keep the
                          one-stage reduction for all; otherwise at least 137 (CDCS_E_ARG).
                          Same projection, other cost.  cdcs_psd_project uses 137. */
} cdcs_settings;

typedef struct {
  int32_t iter;        /* iterations performed so far */
  int32_t status;      /* CDCS_RUNNING ... CDCS_MAX_ITER */
  double eps_p, eps_d, eps_g;   /* relative residuals of the current iterate */
  double obj_p, obj_d;          /* c^T x / tau and b^T y / tau */
  double tau, kappa;
  double cx, by;                /* c^T x and b^T y (certificate scales) */
} cdcs_info;

/* Fill s with eps_tol = 1e-4, max_iter = 2000, check_every = 1, timing = 0,
 * use_graph = 0, eig_fp32 = 0, autotune = 0, alpha = 1, eig_warm = 0,
 * method = CDCS_METHOD_SELF_DUAL, rho = 1, jacobi_max = 0 (automatic), band_min = 0 (automatic). */
void cdcs_default_settings(cdcs_settings* s);

/* Build the cached data of step 1 (the m x m factor of the matrix of eq.
 * FactorizationMatrix after the matrix inversion lemma, and the
 * Sherman-Morrison vector M^{-1} zeta and scalar 1 + zeta^T M^{-1} zeta of
 * eq. MatrixInverseResult), move everything to the GPU and set
 * u = v~ = (0, 0, 0, 0, 1).  `stream` is a hipStream_t or NULL. */
int cdcs_setup(const cdcs_problem* prob, const cdcs_settings* s, void* stream, cdcs_handle** out);

/* The same for `count` independent instances solved together in one
 * launch per phase (prob[count]). */
int cdcs_setup_batch(int32_t count, const cdcs_problem* prob, const cdcs_settings* s,
                     void* stream, cdcs_handle** out);

/* Exactly k ADMM iterations (eqs. Step1-Step3) of every instance, without
 * early exit.  infos (may be NULL) receives one cdcs_info per instance. */
int cdcs_iterate(cdcs_handle* h, int32_t k, cdcs_info* infos);

/* Iterate until every instance has a status other than CDCS_RUNNING (an
 * instance that stops keeps its final iterate while others continue) or
 * max_iter.  infos (may be NULL) receives one cdcs_info per instance. */
int cdcs_solve(cdcs_handle* h, cdcs_info* infos);

/* dims[0..3] = nE, ns, m, p of instance `inst`. */
int cdcs_get_dims(const cdcs_handle* h, int32_t inst, int64_t dims[4]);

/* The nE lower entries (row >= col) of E' in canonical order. */
int cdcs_get_entries(const cdcs_handle* h, int32_t inst, int32_t* row, int32_t* col);

/* Solution of a SOLVED instance (Section 3.2, recovery as in O'Donoghue et
 * al. 2016): X = svec(x)/tau on E' (nE values, canonical order; any PSD
 * completion gives the off-pattern entries, Theorem 1), y/tau (m), and
 * Z = sum_k E_k^T Z_k E_k with Z_k = smat(z_k)/tau (Theorem 2) as svec over
 * E' (nE).  Any output may be NULL.  on_device = 1: outputs are device
 * pointers written on the handle's stream.  CDCS_E_STATE if not solved. */
int cdcs_get_solution(const cdcs_handle* h, int32_t inst, double* X, double* y, double* Z,
                      int32_t on_device);

/* Certificate of an infeasible instance (self-dual method only): PRIMAL_INFEASIBLE gives
 * y_cert = y / b^T y (m) with A^T y_cert + H^T v ~ 0, v ~ z PSD, b^T y_cert = 1
 * (X_cert untouched); DUAL_INFEASIBLE gives X_cert = x / (-c^T x) (nE) with
 * A x ~ 0, H x ~ s PSD, c^T x = -1 (y_cert untouched).  CDCS_E_STATE
 * otherwise. */
int cdcs_get_certificate(const cdcs_handle* h, int32_t inst, double* y_cert, double* X_cert,
                         int32_t on_device);

/* Copy the iterate (u, v~) of instance `inst` out of / into the solver, in
 * the flattened coordinates above (host pointers).  set_state also resets
 * the instance's status to RUNNING; the iteration counter is kept.  With
 * the primal-only / dual-only methods u = (x, s, y) (nE + ns + m values;
 * dual: z in place of s, x the multiplier of step 1) and vt = lam (ns values;
 * dual: lam then v, 2 ns values). */
int cdcs_get_state(const cdcs_handle* h, int32_t inst, double* u, double* vt);
int cdcs_set_state(cdcs_handle* h, int32_t inst, const double* u, const double* vt);

/* Reverse-mode derivative of the solution with respect to the data, through
 * the fixed point of the ADMM iteration (eqs. Step1-Step3 written as
 * z+ = T(z) with z = u - v~; implicit differentiation of z* = T(z*)).
 * dX (NE values: per instance, svec over E' in canonical order, concatenated
 * over instances) is dL/dX for X = x / tau.  Outputs: dC (NE values, dL/dc
 * for c = svec(C), i.e. the gradient with respect to C as an svec) and db
 * (sum of m values, dL/db).  The adjoint system (I - T'^T) mu = g is solved
 * by restarted GMRES(20), one Krylov basis per instance.  An instance stops
 * when ||g - (I - T'^T) mu|| <= tol ||g||, or when that residual has fallen
 * by less than 10% over 5 restarts (the system is singular and consistent
 * only to the accuracy of the forward solve, so the gradient's accuracy
 * follows eps_tol of the solve, not tol); all stop after max_iter operator
 * applications.  *iters (may be NULL) receives the number of applications.
 * on_device = 1: dX, dC, db are device pointers.  Every instance must be
 * SOLVED (CDCS_E_STATE) and have cliques of at most 96 vertices
 * (CDCS_E_ARG): the eigen-cache of the projection's derivative is a Jacobi
 * decomposition held in LDS. */
int cdcs_adjoint(cdcs_handle* h, const double* dX, double* dC, double* db, int32_t on_device,
                 int32_t max_iter, double tol, int32_t* iters);

/* Outcome of the last cdcs_adjoint on this handle, per instance (arrays of
 * the batch's instance count; either may be NULL): resid = the final
 * relative residual ||g - (I - T'^T) mu|| / ||g|| of the adjoint system,
 * reason = 0 if it is within tol, 1 if GMRES stopped because the residual
 * stalled (the gradient is then as accurate as the forward solve allows),
 * 2 if it stopped at max_iter.  The adjoint itself returns 0 in all three
 * cases.  CDCS_E_STATE before the first cdcs_adjoint. */
int cdcs_get_adjoint_info(const cdcs_handle* h, double* resid, int32_t* reason);

/* Accumulated HIP-event time (ms) and launch count per kernel phase since
 * setup or the last reset (timing must be enabled).  names/ms/launches may
 * be NULL; returns the number of phases. */
int cdcs_get_phase_times(const cdcs_handle* h, const char** names, double* ms, int64_t* launches,
                         int32_t cap);
int cdcs_reset_phase_times(cdcs_handle* h);

/* The conic step on its own (eq. Step2, PSD part): project `count` packed
 * symmetric blocks onto their PSD cones, out_k = svec(V max(Lambda,0) V^T)
 * for in_k = svec(V Lambda V^T).  sizes[k] = order of block k (1..1024),
 * offsets[k] = its first element in `in`/`out` (host arrays); in/out are
 * device pointers (may alias).  Runs on `stream` and synchronises it. */
int cdcs_psd_project(int32_t count, const int32_t* sizes, const int64_t* offsets,
                     const double* in, double* out, void* stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same projection
 * as cdcs_psd_project, with the same arguments, kernels and results, but all
 * device memory beyond `in` and `out` (the block index lists and the
 * large-block workspace) lives in a fixed 64 MiB array in the library's
 * device code, one per GPU, held from module load until the process ends.
 * No hipMalloc or hipFree is called.  The current device must be the one
 * `stream` belongs to.  Limit: the index lists (at most 28 bytes per block) plus the
 * large-block workspace (8 (5 l^2 + 5 l + 16 + T(T+1) + 64) bytes per block
 * of order K > 64, l = K rounded up to 8, T = ceil(K/32)) must fit in 64 MiB
 * (e.g. one block of order 1024, or twenty-five of order 256); a larger request
 * returns CDCS_E_ARG without launching anything.  Every call on one GPU uses
 * that GPU's single array, so calls that overlap on one GPU (from two
 * threads, or on two streams without ordering) race; calls ordered on one
 * stream are safe (each clears the workspace it uses before use). */
int cdcs_psd_project_noalloc(int32_t count, const int32_t* sizes, const int64_t* offsets,
                             const double* in, double* out, void* stream);

/* The Jacobi tile shape used per clique-size bucket (the autotuner's choice,
 * or the default): out[4 b + 0..3] = bucket's largest clique order (16, 32,
 * 64, 96), threads per clique, number of cliques in the bucket, 1 if the
 * autotuner measured it.  Returns the number of buckets (4) or an error. */
int cdcs_get_tuning(const cdcs_handle* h, int32_t* out, int32_t cap);

const char* cdcs_last_error(void);
int cdcs_abi_version(void);
void cdcs_destroy(cdcs_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* CDCS_H */
