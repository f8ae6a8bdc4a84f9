/*
 * mx.h -- C ABI of the MI355X (gfx950) time-harmonic Maxwell solver.
 *
 * The library solves, for every transmitting antenna, the lowest-order
 * Nedelec edge-element discretisation of
 *
 *     curl curl E - k0^2 eps_r E = -j omega mu0 J          in Omega,
 *     (curl E) x n + j k n x (E x n) = 0                   on dOmega,
 *
 * (time factor exp(+j omega t), k = k0 sqrt(eps_r)); this is the forward
 * problem of the microwave-imaging method (paper Sec. IV-B, eq. (1) and
 * its weak form (2), with the open-side impedance condition on the whole
 * outer boundary and point dipoles in place of the waveguide ports).  The
 * linear systems A u_j = b_j (Sec. IV-C) are solved with right-
 * preconditioned flexible GMRES and a one-level Optimized Restricted Additive
 * Schwarz preconditioner (Sec. IV-C), with all transmitters as one block of
 * right-hand sides.  Receiver responses S_ij = r_i^T u_j follow the
 * scattering functional (eq. (3)) with point receivers.
 *
 * Conventions
 *   - Every function returns an int: MX_OK (0) on success, a negative MX_E*
 *     code on failure; mx_last_error() then returns a message (thread-local,
 *     valid until the next call on the same thread).  No C++ exception
 *     crosses this boundary.
 *   - Units are SI (metres, hertz).  eps_r is dimensionless complex with
 *     negative imaginary part for lossy media.
 *   - Complex numbers are interleaved (re, im) pairs of doubles (mx_c128).
 *   - Block vectors are DOF-major: X[e * nrhs + j] is DOF (edge) e of
 *     right-hand side j.
 *   - Pointers marked "host or device" may point to host memory or to
 *     device memory of the context's GPU; the library detects which.  All
 *     other pointers are host memory.  The caller owns every buffer it passes;
 *     the library copies inputs before returning.
 *   - A context is not thread-safe.  Work runs on the context's stream and
 *     every call synchronises before returning.
 *   - Call order: mx_create -> mx_assemble -> mx_setup_schwarz -> mx_solve...
 *     mx_assemble invalidates the Schwarz factors (call mx_setup_schwarz
 *     again); out-of-order calls return MX_ESTATE.
 */
#ifndef MX_H
#define MX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MX_OK = 0,
  MX_EINVAL = -1,   /* invalid argument (sizes, NaN permittivity, inverted tet, point outside) */
  MX_ENOMEM = -2,   /* device or host allocation failed */
  MX_ESTATE = -3,   /* call out of order */
  MX_ENOTCONV = -4, /* FGMRES hit maxit; outputs hold the last iterate */
  MX_EPIVOT = -5,   /* zero pivot in a subdomain factorisation */
  MX_EHIP = -6      /* HIP runtime error */
};

enum { MX_EPS_P0 = 0 /* one value per tetrahedron */, MX_EPS_P1 = 1 /* one value per vertex */ };
enum { MX_PREC_C128 = 0 /* complex128 subdomain factors */, MX_PREC_C64 = 1 /* complex64 factors on MFMA */ };

typedef struct mx_ctx mx_ctx;

typedef struct { double re, im; } mx_c128;

/* Tetrahedral mesh: xyz [nv][3] coordinates, tet [nt][4] 0-based vertex ids
 * (any orientation).  Global edges are the distinct (vmin, vmax) vertex pairs
 * numbered in lexicographic order; they are the unknowns. */
typedef struct {
  int32_t nv, nt;
  const double* xyz;
  const int32_t* tet;
} mx_mesh;

/* Options of the Schwarz preconditioner and the Krylov solver. */
typedef struct {
  int32_t precision;   /* MX_PREC_C128 or MX_PREC_C64 */
  int32_t restart;     /* FGMRES restart length m (default 15 when <= 0) */
  int32_t maxit;       /* iteration cap (default 2000 when <= 0) */
  int32_t factor;      /* 1: factor the subdomain matrices (normal use);
                          0: keep them assembled (mx_get_local_matrix only) */
  int32_t coarse;      /* 1: add the learned coarse correction (needs weights:
                          mx_coarse_init / mx_coarse_set_weights); 0: one-level ORAS */
} mx_schwarz_opts;

/* Point dipoles: pos [n][3] positions, moment [n][3] complex moments (A m).
 * A unit z-dipole has moment (0,0,1). */
typedef struct {
  int32_t n;
  const double* pos;
  const mx_c128* moment;
} mx_sources;

/* Waveguide port (Sec. IV-B, eq. (1)): a planar rectangle on the mesh
 * boundary with outward unit normal `normal`, broad-side direction `u`
 * (orthogonalised against the normal), width a along u and height b along
 * v = normal x u, centred at `centre`, filled with relative permittivity eps.
 * Its TE10 profile is e(x) = sin(pi (s + a/2) / a) v, s = (x - centre).u,
 * and beta = sqrt(k0^2 eps - (pi/a)^2) with Im beta <= 0. */
typedef struct {
  double centre[3];
  double normal[3];
  double u[3];
  double a, b;
  mx_c128 eps;
} mx_port;

/* Per-solve diagnostics (arrays are caller-owned, length nrhs, may be NULL). */
typedef struct {
  int32_t* iters;      /* Krylov iterations per right-hand side */
  double* relres;      /* final true relative residual ||b - A x|| / ||b|| */
  int32_t iters_max;   /* max over right-hand sides */
  int32_t cycles;      /* restart cycles */
  double t_iter;       /* seconds spent in the Krylov iteration */
  int32_t fallback;    /* 1/2/3: the learned coarse term was switched off during the
                          solve (non-finite output / a cycle with < 10% reduction /
                          the first steps removed < 5% of the one-level residual);
                          4: block FGMRES fell back to the pseudo-block solver */
  double t_assemble;   /* seconds of the mx_assemble that built the operator in use
                          (operator values; includes topology when a mesh was given) */
  double t_setup;      /* seconds of the mx_setup_schwarz that built the factors in use
                          (local matrices + factorisation; partition when rebuilt) */
  double t_lu;         /* of t_setup: device time of the batched factorisation */
} mx_solve_info;

/* Sizes of the current discretisation and decomposition. */
typedef struct {
  int64_t nv, nt, ne, nnz, nbface;
  int32_t nsub, overlap, ncolour;
  int64_t sum_ni;      /* sum of subdomain DOF counts n_i */
  int64_t sum_Ni2;     /* sum of padded dense sizes N_i^2 (factor entries) */
  int32_t nb;          /* dense block size; N_i = n_i rounded up to nb */
  /* Work of the banded factorisation and solves (0 before a factorisation):
   * the subdomain unknowns are kept in reverse Cuthill-McKee order, so the
   * dense local matrices are banded and only 64x64 tiles inside the band are
   * visited. */
  int64_t lu_tiles;          /* 64x64x64 complex tile products of the trailing updates */
  int64_t trsm_tiles_lower;  /* 64x64 factor tiles read by one forward solve (all subdomains) */
  int64_t trsm_tiles_upper;  /* 64x64 factor tiles read by one backward solve */
} mx_sizes;

/* Kernel classes timed by mx_set_profiling / mx_get_kernel_times. */
enum {
  MX_K_LU_PANEL = 0,    /* panel factorisation (one launch per 64 columns)   */
  MX_K_LU_ROWPANEL = 1, /* row interchanges + U12 block row                  */
  MX_K_LU_UPDATE = 2,   /* trailing-matrix update A22 -= L21 U12 (MFMA)       */
  MX_K_LU_INV = 3,      /* diagonal-block inversion + permutation            */
  MX_K_TRSM_LOWER = 4,  /* batched multi-RHS forward solve (MFMA)            */
  MX_K_TRSM_UPPER = 5,  /* batched multi-RHS backward solve (MFMA)           */
  MX_K_SPMM = 6,        /* complex CSR block SpMM                           */
  MX_K_RESTRICT = 7,    /* restriction R_i (gather + cast)                  */
  MX_K_PROLONG = 8,     /* prolongation sum_i R_i^T D_i (all colours)         */
  MX_K_CGS = 9,         /* classical Gram-Schmidt x2 + norm + Givens, per step */
  MX_K_ASSEMBLE = 10,   /* element/face blocks + CSR gather                  */
  MX_K_LOCAL = 11,      /* dense subdomain assembly (zero fill + gather)     */
  MX_K_COARSE = 12,     /* learned coarse correction (pooling, network, prolongation) */
  MX_K_NCLASS = 16
};
typedef struct {
  double ms[MX_K_NCLASS];       /* summed device time per class (milliseconds) */
  int64_t launches[MX_K_NCLASS]; /* number of timed intervals per class         */
} mx_kernel_times;

/* Create a context on HIP device `device`.  hip_stream (a hipStream_t passed
 * as void*) is the stream all work of the context runs on; NULL gives the
 * context a stream of its own.  The caller keeps a passed stream alive while
 * the context uses it.  Errors: MX_EINVAL (NULL out, no such device), MX_EHIP. */
int mx_create(mx_ctx** out, int device, void* hip_stream);
int mx_destroy(mx_ctx* ctx);

/* Run all further work of the context on the caller's HIP stream
 * (hipStream_t passed as void*; NULL returns to the context's own stream).
 * The caller keeps the stream alive while the context uses it. */
int mx_set_stream(mx_ctx* ctx, void* hip_stream);

/* Autotuner (on by default): at the first solve of a problem shape (edges,
 * non-zeros, subdomains, factor entries, precision, number of right-hand
 * sides) the candidate variants below are timed on the problem's own data
 * with HIP events and the fastest is used from then on:
 *   SpMM: 0 = one lane per right-hand side, non-zeros read by every lane;
 *         1 = 32 lanes per row, each non-zero read once and broadcast
 *             (nrhs <= 32 only);
 *         2 = column windows: slices of at most 32 consecutive rows whose
 *             non-zeros touch at most 128 columns; each workgroup stages
 *             its slice's X rows (16 right-hand sides) in LDS once and
 *             forms the slice's rows from there (built with the mesh;
 *             unavailable when a row has more than 128 non-zeros);
 *   triangular solves: workgroup order (1 = b-th largest subdomain paired
 *         with the b-th smallest, 0 = largest first) x right-hand-side
 *         columns per workgroup (32, or 16 with twice the workgroups and
 *         four resident per compute unit).
 * and, at the first factorisation (mx_setup_schwarz) of a shape bucket
 * (precision, subdomain count, largest subdomain / 4096 unknowns):
 *   factorisation: panels per trailing-update pass of the banded LU
 *         (1, 2, 4 or 8), each timed on a whole factorisation of the
 *         problem's own local matrices (the set-up then factors once more
 *         with the fastest).
 * Tuning cache: when the environment variable MX_TUNE_CACHE names a file,
 * results are looked up there first (a hit skips the timing) and new ones
 * are added to it; the file is a JSON object, one entry per line, keyed by
 * "solve:<hash of the problem shape>" and "lu:<precision>:<subdomains>:
 * <largest subdomain / 4096>", written through a temporary file and a rename.
 * enable = 0 switches it off and restores variant 0 / paired order / 32 /
 * two panels per pass. */
typedef struct {
  int32_t spmm_variant;
  int32_t trsm_paired;
  int32_t trsm_cols;
  double spmm_ms[3];   /* average time of one SpMM per variant (0 if not run,
                          1e30 if the variant does not apply)               */
  double trsm_ms[4];   /* one lower + upper solve: [largest first / 32 columns,
                          paired / 32, largest first / 16, paired / 16]      */
  int32_t lu_group;    /* panels per trailing-update pass of the factorisation */
  double lu_ms[4];     /* one factorisation with 1, 2, 4, 8 panels per pass
                          (0 if not timed)                                   */
  int32_t from_cache;  /* bit 0: SpMM / solve variants, bit 1: panel group,
                          taken from the tuning cache                        */
} mx_tuning;
int mx_set_autotune(mx_ctx* ctx, int enable);
/* Fix the factorisation's panels per trailing-update pass (1..16; the
 * factors differ only by rounding), or 0 to let the autotuner pick it again.
 * Takes effect at the next mx_setup_schwarz. Errors: MX_EINVAL. */
int mx_set_lu_group(mx_ctx* ctx, int32_t group);
/* Fix the variants (switches the autotuner off): spmm_variant 0/1/2,
 * trsm_paired 0/1, trsm_cols 16/32. Results do not depend on the variants
 * beyond rounding. Errors: MX_EINVAL. */
int mx_set_tuning(mx_ctx* ctx, int32_t spmm_variant, int32_t trsm_paired, int32_t trsm_cols);
int mx_get_tuning(mx_ctx* ctx, mx_tuning* out);

/* Krylov solver of every solve (mx_solve, mx_solve_rhs, mx_solve_ports and
 * the adjoint solve of mx_gradient), Sec. IV-C:
 *   MX_KRYLOV_PSEUDO_BLOCK (default): one FGMRES per right-hand side, run as
 *     one block of kernels;
 *   MX_KRYLOV_BLOCK: block FGMRES, one block Krylov space shared by all
 *     right-hand sides: block Arnoldi with one pass of classical block
 *     Gram-Schmidt (a second pass only when the pass removed all but 1e-8
 *     of a column's squared norm), the new block orthonormalised by Cholesky
 *     QR (a second pass unless the block is well conditioned); block
 *     Hessenberg least squares by Givens rotations on the host;
 *   MX_KRYLOV_BLOCK_CGS2: the same with block Gram-Schmidt applied twice and
 *     Cholesky QR applied twice (more robust, more sweeps over the basis).
 *   Both block modes: one-level preconditioner; with the learned term set up
 *     (coarse = 1), a solve starts with the pseudo-block solver and the
 *     judged learned term and continues with block FGMRES from the current
 *     iterate once the judge has switched the term off; restart after
 *     `restart` block steps,
 *     every right-hand side to the same rtol of its own ||b_j||. More than 32
 *     right-hand sides are split into balanced groups of at most 32, each
 *     with its own block Krylov space; the groups advance in lockstep (one
 *     preconditioner and operator application over the whole width). With a
 *     zero right-hand side, or a residual block of numerical rank below its
 *     width at the start, the solve runs the pseudo-block solver instead and
 *     reports fallback = 4. Iteration counts are block steps of the
 *     right-hand side's group.
 * Errors: MX_EINVAL (unknown mode). */
enum { MX_KRYLOV_PSEUDO_BLOCK = 0, MX_KRYLOV_BLOCK = 1, MX_KRYLOV_BLOCK_CGS2 = 2 };
int mx_set_krylov(mx_ctx* ctx, int32_t mode);

/* Port form of the boundary conditions of eq. (1) (Sec. IV-B). A boundary
 * face belongs to port p when its centroid lies in that port's plane and
 * rectangle (relative tolerance 1e-6 of a + b); port faces carry
 * j beta_p int (E x n).(v x n) in place of the impedance term. With pec != 0
 * every other boundary face is a metallic wall (n x E = 0): its edges are
 * eliminated symmetrically (row and column cleared, diagonal 1, zero
 * right-hand side) in the operator and in the subdomain matrices; with
 * pec == 0 they keep the impedance condition. Needs a mesh (mx_assemble);
 * re-assembles the operator values; mx_setup_schwarz must follow.
 * nports = 0 restores the impedance boundary everywhere. A new mesh clears
 * the ports. Errors: MX_EINVAL (bad sizes or non-finite data), MX_ESTATE. */
int mx_set_ports(mx_ctx* ctx, int32_t nports, const mx_port* ports, int32_t pec);

/* All-port solve (eqs. (1), (3)): transmitter p is the TE10 incidence
 * g = 2 j beta_p e_p on port p (b_e = int g.N_e over the port), all ports as
 * one block right-hand side, FGMRES to relative true residual rtol;
 * S[i][j] = int_{port i} E_j.e_i / int_{port i} e_i.e_i - delta_ij.
 *   E [ne][nports] (host or device, may be NULL), S [nports][nports].
 * Returns MX_ENOTCONV (outputs written) when maxit is reached. */
int mx_solve_ports(mx_ctx* ctx, double rtol, mx_c128* E, mx_c128* S, mx_solve_info* info);

/* enable != 0 (the default): Arnoldi steps that use the one-level
 * preconditioner are captured as HIP graphs and replayed. A step runs eagerly
 * the first time it is reached with the current buffers, sizes and
 * tolerance; from the second time on it is one graph launch. Steps with the
 * learned term, and all steps while profiling is on, run eagerly.
 * enable = 0 drops the captured graphs. Results are bitwise identical. */
int mx_set_graphs(mx_ctx* ctx, int enable);

/* enable != 0: bracket every launch of the classes above with HIP events on
 * the context's stream (small overhead) and reset the totals; 0: stop. */
int mx_set_profiling(mx_ctx* ctx, int enable);
/* Totals since profiling was enabled (synchronises the stream). */
int mx_get_kernel_times(mx_ctx* ctx, mx_kernel_times* out);

/* Operator assembly (eq. (2)): A = sum_T (K_T - k0^2 eps M_T) + j k_b sum_F B_F
 * over the tetrahedra T and the outer boundary faces F, k_b = k0 sqrt(eps_b).
 *   mesh      host; NULL reuses the mesh (topology) of the previous call
 *   eps       [nt] (MX_EPS_P0) or [nv] (MX_EPS_P1) relative permittivity;
 *             host or device
 *   freq_hz   frequency (> 0)
 *   eps_b     permittivity used in the outer impedance condition
 * Tetrahedra may have either orientation (vertex ids are sorted and |det|
 * is used).
 * Errors: MX_EINVAL for bad sizes, a frequency that is not positive (k0 = 0
 * would leave the curl-curl operator singular), non-finite eps or a
 * degenerate (zero-volume) tet. */
int mx_assemble(mx_ctx* ctx, const mx_mesh* mesh, const mx_c128* eps, int eps_kind,
                double freq_hz, mx_c128 eps_b);

/* ORAS set-up (Sec. IV-C): recursive coordinate bisection into nsub = 2^L
 * parts, `overlap` layers of vertex-adjacent tetrahedra, integer partition
 * of unity, local matrices with impedance transmission conditions, and the
 * batched dense LU of all subdomain matrices (one set of launches).  The
 * partition is cached while the mesh, nsub and overlap are unchanged.
 * opts may be NULL (complex128, restart 15, maxit 2000, factor 1).
 * Errors: MX_EINVAL (nsub not a power of two, overlap < 1), MX_EPIVOT (a
 * subdomain matrix has a column with no usable pivot: zero or non-finite,
 * e.g. entries beyond the complex64 range; the message names the subdomain
 * and the column; the factors are not usable and solves return MX_ESTATE). */
int mx_setup_schwarz(mx_ctx* ctx, int32_t nsub, int32_t overlap, const mx_schwarz_opts* opts);

/* All-transmitter solve: b_j = -j omega mu0 p_j . N_e(x_j) for every source
 * (a point on a shared face/edge/vertex averages over its tetrahedra), block
 * FGMRES to relative true residual rtol, receiver responses
 * S[i][j] = p_i . E_j(x_i) for the receivers rx (NULL: rx = tx).
 *   E  [ne][ntx] fields, host or device, may be NULL
 *   S  [nrx][ntx] host or device, may be NULL
 * Returns MX_ENOTCONV (outputs still written) when maxit is reached;
 * MX_EINVAL for an empty source set, more than 256 transmitters or a point
 * outside the mesh. */
int mx_solve(mx_ctx* ctx, const mx_sources* tx, const mx_sources* rx, double rtol,
             mx_c128* E, mx_c128* S, mx_solve_info* info);

/* Cost and adjoint-state gradient of the inverse problem (Sec. IV-D, eq. (4)):
 *   J = 1/2 sum_ij w_ij |S_ij - S_meas_ij|^2 + alpha/2 int |grad kappa|^2,
 *   kappa = k0^2 eps, eps piecewise linear (MX_EPS_P1),
 * for the transmitters and receivers of the immediately preceding mx_solve
 * (same operator and factors).  The adjoint fields solve A lambda_j =
 * sum_i w_ij conj(d_ij) r_i with the same preconditioner (A is complex
 * symmetric), and
 *   grad_n = dJ/dRe eps_n + j dJ/dIm eps_n
 *          = conj(k0^2 sum_j lambda_j^T M_n u_j) + alpha k0^4 (K1 eps)_n,
 * M_n = int lambda_n N_e . N_f, K1 the P1 stiffness matrix.
 *   S_meas [nrx][ntx] host;  w [nrx][ntx] host weights (1/|S_empty|^2, 0 on
 *   entries to ignore);  grad [nv] host or device;  J host;  info may be NULL
 *   (adjoint iteration counts).
 * Errors: MX_ESTATE without a preceding mx_solve, MX_EINVAL for per-tetrahedron
 * permittivity or a negative alpha. */
int mx_gradient(mx_ctx* ctx, const mx_c128* S_meas, const double* w, double alpha, mx_c128* grad, double* J,
                mx_solve_info* info);

/* Same solver on caller-supplied right-hand sides b [ne][nrhs] (host or
 * device); solution x [ne][nrhs] (host or device). */
int mx_solve_rhs(mx_ctx* ctx, const mx_c128* b, int32_t nrhs, double rtol,
                 mx_c128* x, mx_solve_info* info);

/* Y = A X for X, Y [ne][nrhs] (host or device). */
int mx_apply_operator(mx_ctx* ctx, const mx_c128* X, mx_c128* Y, int32_t nrhs);

/* Z = M^{-1} X = sum_i R_i^T D_i B_i^{-1} R_i X (one ORAS application;
 * complex64 factors round R_i X to complex64).  X, Z host or device.
 * With the learned term set up (opts.coarse = 1 and weights), Z is the
 * preconditioner FGMRES applies: Z_j = M^{-1} X_j + theta_j q_j, q the
 * learned correction and theta_j minimising ||X_j - A Z_j||_2. */
int mx_apply_preconditioner(mx_ctx* ctx, const mx_c128* X, mx_c128* Z, int32_t nrhs);

/* Allocation-free variant of mx_apply_preconditioner, for callers that cannot
 * allocate device memory (tight serving loops, code that must not call
 * hipMalloc). Z = M^{-1} X with the one-level preconditioner only (the
 * learned term needs allocated buffers: MX_ESTATE when it is set up).
 *   X, Z  device pointers [ne][nrhs] on the context's GPU, owned by the
 *         caller (X == Z allowed).
 * The restricted vectors live in a fixed device array of 64 MiB (each GPU
 * the library runs on holds its own until the process ends); a call needs
 * sum_i N_i * nrhs * (16 bytes complex128 / 8 bytes complex64) of it and
 * returns MX_EINVAL beyond that (e.g. the 1.02M-edge chamber with 512
 * subdomains: 21 MB per right-hand side with complex64 factors, so at most
 * 3 per call). The call allocates nothing and does not synchronise: the work
 * is enqueued on the context's stream and Z is ready when the stream has
 * executed it. All contexts on one GPU share the array, so calls whose work
 * overlaps on one GPU (two streams, two threads) race; calls in one stream
 * are ordered. Errors: MX_EINVAL (sizes, host pointers), MX_ESTATE. */
int mx_apply_preconditioner_noalloc(mx_ctx* ctx, const mx_c128* X, mx_c128* Z, int32_t nrhs);

/* Sizes of the current state (zeros for parts not yet built). */
int mx_get_sizes(mx_ctx* ctx, mx_sizes* out);

/* Copies of the topology (host buffers of the sizes in mx_sizes; any may be
 * NULL): edges [ne][2], t2e [nt][6] (edges of the id-sorted tetrahedron in
 * the order (01,02,03,12,13,23)), row_ptr [ne+1], col [nnz]. */
int mx_get_topology(mx_ctx* ctx, int32_t* edges, int32_t* t2e, int64_t* row_ptr, int32_t* col);

/* Copy of the assembled CSR values [nnz] (host). */
int mx_get_matrix_values(mx_ctx* ctx, mx_c128* val);

/* Copies of the decomposition (host, any may be NULL): part [nt] core
 * subdomain of each tetrahedron, dof_ptr [nsub+1], dofs [sum_ni] (sorted
 * global edges of each overlapping subdomain), pu_w [sum_ni] integer
 * partition-of-unity weights, colour [nsub]. */
int mx_get_partition(mx_ctx* ctx, int32_t* part, int64_t* dof_ptr, int32_t* dofs,
                     int32_t* pu_w, int32_t* colour);

/* Copy of the assembled (unfactored, opts.factor = 0) local matrix of
 * subdomain i as a dense row-major [n_i][n_i] array (host). */
int mx_get_local_matrix(mx_ctx* ctx, int32_t i, mx_c128* B);

/* Point functionals r[e] = p . N_e(x) of the given points as a dense
 * [ne][n] array (host); the same values build right-hand sides. */
int mx_point_functionals(mx_ctx* ctx, const mx_sources* pts, mx_c128* R);

/* ---- learned coarse-space correction -------------------------------------
 * An additive correction to the one-level ORAS preconditioner (not in the
 * paper; the solver's own addition): for a block v, features
 * x_i = P_i^T R_i v / s (s = ||v|| / sqrt(ne) per column; P_i the 4x4x4
 * lattice prolongation of subdomain i, 192 complex = 384 real channels),
 * a per-subdomain network (MLP 384-256-256-256-256 with GELU, two message-
 * passing layers over subdomain adjacency, 384 outputs) with bf16 operands and
 * FP32 accumulation, and q = s * out_scale * sum_i R_i^T D_i P_i c_i added to
 * M^{-1} v.  FGMRES tolerates the nonlinear preconditioner; the solver falls
 * back to plain ORAS on non-finite output or a stagnating cycle.
 * Parameters: flat FP32 vector of mx_coarse_num_params() values in the order
 * W1 b1 W2 b2 W3 b3 W4 b4 Ws1 Wn1 b5 Ws2 Wn2 b6 (W row-major [out][in]);
 * inputs are divided by in_scale, outputs multiplied by out_scale. */
int64_t mx_coarse_num_params(void);
/* Random initial weights (seeded; normal, 1/fan_in variance, output layers x0.1). */
int mx_coarse_init(mx_ctx* ctx, uint64_t seed);
/* Set the parameters (n = mx_coarse_num_params()) and scales; resets the
 * Adam moments and step count. */
int mx_coarse_set_weights(mx_ctx* ctx, const float* theta, int64_t n, double in_scale, double out_scale);
int mx_coarse_get_weights(mx_ctx* ctx, float* theta, int64_t n, double* in_scale, double* out_scale);
/* Pooled features X [nrhs][nsub][384] (host) of v [ne][nrhs] (host or device). */
int mx_coarse_features(mx_ctx* ctx, const mx_c128* v, int32_t nrhs, float* X);
/* Network outputs out [ngraph][nsub][384] for inputs X [ngraph][nsub][384]
 * (host; scales not applied). */
int mx_coarse_forward(mx_ctx* ctx, const float* X, int32_t ngraph, float* out);
/* Network outputs as mx_coarse_forward, and the hidden activations
 * H [5][ngraph][nsub][256] (host): the four MLP layers and the first
 * message-passing layer, after GELU. */
int mx_coarse_hidden(mx_ctx* ctx, const float* X, int32_t ngraph, float* H, float* out);
/* Mean squared error against Y and its parameter gradient (host buffers). */
int mx_coarse_loss_grad(mx_ctx* ctx, const float* X, const float* Y, int32_t ngraph, double* loss, float* grad);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) of the
 * FP32 master weights with the given gradient grad [n] (host or device,
 * n = mx_coarse_num_params()), e.g. a gradient averaged over several
 * processes; mx_coarse_train uses the same update. */
int mx_coarse_adam_step(mx_ctx* ctx, const float* grad, int64_t n, double lr);
/* Training data from the plain solver on the current operator: solves the
 * transmitters to rtol_exact, then re-runs with restart length snap_every and
 * records, at every restart, the features of the residual r and the
 * least-squares lattice fit of R_i (e - M^{-1} r)/s (e = exact - current
 * iterate), up to max_snapshots restarts; appends to the context's data set. */
int mx_coarse_collect(mx_ctx* ctx, const mx_sources* tx, int32_t snap_every, int32_t max_snapshots,
                      double rtol_exact, int32_t* nsnap);
int mx_coarse_clear(mx_ctx* ctx);
/* Adam on the collected data (mean squared error in scaled units), batches of
 * batch_graphs (snapshot, transmitter) graphs; loss_hist [epochs] may be NULL. */
int mx_coarse_train(mx_ctx* ctx, int32_t epochs, int32_t batch_graphs, double lr, uint64_t seed, double* loss_hist);

const char* mx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MX_H */
