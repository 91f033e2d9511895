/*
 * ddamg.h - C ABI of the MI355X (gfx950) multi-rhs x multi-shift twisted-mass
 * DD-alpha-AMG solver.
 *
 * Method: Yamamoto, Bacchio, Finkenrath, "Implementation of Simultaneous
 * Inversion of a Multi-shifted Dirac Matrix for Twisted-Mass Fermions within
 * DDalphaAMG" (arXiv:2201.03872).  Section 1/3: many right-hand sides and many
 * twisted-mass values are inverted simultaneously; section 2: the
 * preconditioner is red-black SAP plus aggregation-based coarse-grid
 * correction, recursive over levels; section 4: FGMRES at the top level to a
 * 1e-10 goal residual, FGMRES / (block) GMRES on the coarse levels; Fig. 6
 * caption: D_TM = D_W + i (delta mu) mu gamma5.
 *
 * Operator (every column c has its own twisted mass mu_c):
 *   D(mu) psi(x) = (4 + m0) psi(x) + i mu gamma5 psi(x)
 *                  - 1/2 sum_nu [ (1 - gamma_nu) U_nu(x) psi(x+nu)
 *                               + (1 + gamma_nu) U_nu(x-nu)^dag psi(x-nu) ]
 *   m0 = 1/(2 kappa) - 4; periodic in x, y, z; antiperiodic in t (the sign
 *   multiplies the hop across the t boundary and is never folded into links).
 *   Chiral gamma basis: gamma_k = [[0,-i s_k],[i s_k,0]], gamma_4 = [[0,1],[1,0]],
 *   gamma5 = diag(1,1,-1,-1).
 *
 * Canonical layouts at this boundary (the "one vector after the other"
 * layout of the paper's Fig. 2, left; the library converts once per call to
 * its internal column-tiled layout, never per operator application inside a
 * solve):
 *   site index      i = x + Lx*(y + Ly*(z + Lz*t)),   mu = 0..3 = x,y,z,t
 *   gauge           double [V][4 mu][3 row][3 col][re,im]; U[x][mu] links x -> x+mu
 *   fine vectors    double [col][V][4 spin][3 colour][re,im]
 *   coarse vectors  double [col][Vc][2N][re,im]    (level l > 0; Vc in the
 *                   lexicographic order of the coarse lattice, coarse dof
 *                   index = chirality*N + j, chirality 0 = gamma5 +1)
 *   coarse blocks   double [Vc][9][2N row][2N col][re,im]; slot 0 = self block
 *                   (without the twist), 1+nu = hop to a+nu, 5+nu = hop to a-nu
 *   solve columns   col = r*n_shift + k  for rhs r and shift k.
 *
 * Memory: every vector argument (x, y, b, f) is a DEVICE pointer on the
 * context's HIP stream (e.g. a torch tensor's data_ptr() on torch's current
 * stream); mu arrays, blocks and test vectors are HOST pointers.  The caller
 * owns every array; the library copies the gauge field at setup and owns the
 * context until ddamg_destroy.  One context per host thread.
 *
 * Errors: 0 on success; negative values are errors (no exception crosses the
 * ABI); +1 = DDAMG_NOT_CONVERGED (the solution is written and per-column
 * residuals are reported).  ddamg_strerror returns a static string.
 */
#ifndef DDAMG_H
#define DDAMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DDAMG_OK             0
#define DDAMG_NOT_CONVERGED  1
#define DDAMG_EINVAL        -1   /* bad dimensions, blocks, levels, NaN input, bad pointer */
#define DDAMG_ENOMEM        -2   /* device allocation failed                              */
#define DDAMG_EDEVICE       -3   /* HIP runtime error                                      */
#define DDAMG_EBREAKDOWN    -4   /* unrecoverable Krylov breakdown                         */
#define DDAMG_ESTATE        -5   /* requested level / object not built                     */

/* arithmetic of one operator application */
#define DDAMG_FP64 0
#define DDAMG_FP32 1
#define DDAMG_FP16 2   /* ddamg_apply_sap only: FP32 SAP reading FP16-stored right-hand sides */

/* solver precision mode */
#define DDAMG_PLAIN_FP64 0   /* everything in FP64                                            */
#define DDAMG_MIXED      1   /* FP64 outer FGMRES; FP32 preconditioner (SAP, R/P, coarse)       */

/* fine-level smoother */
#define DDAMG_SMOOTHER_SAP     0
#define DDAMG_SMOOTHER_LEARNED 1

typedef struct ddamg_ctx ddamg_ctx;

typedef struct ddamg_params {
  int    dims[4];            /* Lx, Ly, Lz, Lt                                                  */
  double kappa;              /* m0 = 1/(2 kappa) - 4                                            */
  int    n_levels;           /* 1 (SAP-preconditioned FGMRES), 2 or 3                           */
  int    agg[2][4];          /* aggregate extents of each level transition                      */
  int    n_tv[2];            /* test vectors N of each level transition (coarse dof = 2N)       */
  int    sap_block[4];       /* SAP block extents; must equal agg[0] when n_levels > 1          */
  int    sap_cycles;         /* red-black SAP cycles per smoother call                          */
  int    sap_mr_iters;       /* MR iterations per block solve                                   */
  int    setup_rounds;       /* smoothing rounds of the random setup vectors                    */
  int    setup_coarse_iters; /* fixed GMRES length per coarse setup round                       */
  int    setup_boot;         /* bootstrap rounds: fine test vectors <- MG cycle(test vectors)   */
  int    setup_fine_iters;   /* 0: fine setup rounds are SAP calls; k > 0: k steps of           */
                             /* SAP-preconditioned FGMRES (inverse iteration)                   */
  double mu_setup;           /* twisted mass used while building the hierarchy                  */
  double coarse_mu_factor;   /* delta mu on the coarsest level (Fig. 6 caption); 1 = none       */
  double tol;                /* outer relative residual goal (1e-10)                            */
  double r_m;                /* middle-level relative tolerance (7e-2)                          */
  double r_b;                /* bottom relative tolerance (1e-1)                                */
  int    outer_restart;      /* FGMRES restart length at the top level                          */
  int    max_outer;          /* cap on outer iterations                                         */
  int    inner_iters;        /* > 0: each outer step preconditions with an FP32 FGMRES of up to */
                             /* this many steps (restart 63) around the MG cycle / smoother;     */
                             /* 0: the MG cycle / smoother alone                                 */
  double inner_tol;          /* relative residual at which that inner FGMRES stops early        */
  int    inner_fp16;         /* 1: that inner FGMRES keeps its Arnoldi basis in FP16 (scaled)   */
  int    middle_restart;     /* FGMRES restart on the middle level                              */
  int    middle_maxit;       /* cap on middle-level iterations per call                         */
  int    bottom_maxit;       /* cap on bottom iterations per call                               */
  int    coarse_smooth_iters;/* MR steps of the middle-level post-smoother                      */
  int    coarsest_block;     /* 1: block GMRES per shift group on the coarsest level            */
  int    precision;          /* DDAMG_PLAIN_FP64 or DDAMG_MIXED                                 */
  int    smoother;           /* DDAMG_SMOOTHER_SAP or DDAMG_SMOOTHER_LEARNED                    */
  int    smoother_cycles;    /* learned smoother: minimal-residual steps along f(r) per call    */
  int    col_tile;           /* columns per tile of the internal layout (4, 8 or 16; 0 = 8)     */
  int    use_graphs;         /* 1: unpreconditioned (coarsest-level) GMRES runs its Arnoldi     */
                             /* steps as captured HIP graphs with device-side least squares    */
  int    max_active_cols;    /* outer solve: columns in flight at once (0 = as memory allows);  */
                             /* the others wait and join as converged columns leave             */
  uint64_t seed;             /* counter-based RNG seed of the setup vectors when none are given */
  int    verbose;            /* 0 = silent                                                      */
  double csw;                /* clover coefficient c_sw of the site term c_sw (i/4) sum          */
                             /* sigma_{mu nu} F_{mu nu} (clover-leaf F); 0 = no clover term       */
  int    sap_oddeven;        /* 1: SAP block solves run MR on the odd-even reduced block systems */
                             /* (4^4 blocks, c_sw = 0); 0: MR on the full block systems         */
  int    coarse_gamma5;      /* Krylov solves of the MG cycle on the gamma5-Hermitian form      */
                             /* gamma5_c D_c(mu) = Q_c + i dmu mu (same solution, same residual */
                             /* norm; the shifted-Hermitian operator is normal): 0 = off,       */
                             /* 1 = the coarsest level, 2 = every coarse level                  */
  int    bottom_restart;     /* restart length m of the coarsest-level GMRES (0: min(bottom_maxit, */
                             /* 63))                                                             */
  int    bottom_dr_k;        /* > 0: the coarsest level runs GMRES with deflated restarting,    */
                             /* GMRES-DR(m, k) (section 4): k harmonic Ritz vectors carried     */
                             /* over each restart; 0 = plain restarted GMRES                     */
  int    coarse_fp16;        /* 1: the Krylov bases of the coarse levels' solves (MIXED       */
                             /* precision) are stored in FP16 like the inner FGMRES basis      */
                             /* (unnormalised, per-column entry scales), halving the bytes of   */
                             /* their Gram-Schmidt passes; such solves run host-driven steps   */
  int    transfer_fp16;      /* 1: the FP32 restriction and prolongation between the fine     */
                             /* level and level 1 read P in FP16 (half the bytes of the        */
                             /* largest array they stream; entries of the orthonormal P are    */
                             /* about 1/sqrt(6 |aggregate|), far inside the FP16 range)        */
} ddamg_params;

typedef struct ddamg_col_info {
  int    outer_iters;        /* outer FGMRES iterations this column took                        */
  int    converged;          /* 1 if the FP64 true residual met tol                             */
  double true_rel_res;       /* ||b - D(mu) x|| / ||b|| in FP64 on the GPU when the column left */
  double err_vs_fp64;        /* the same in an independent FP64 pass after the solve: the       */
                             /* caller's x and b read back from the canonical arrays, r = b -  */
                             /* D(mu) x with the FP64 stencil and links, ||r|| / ||b||; the     */
                             /* result's error against the FP64 operator whatever the precision */
                             /* the preconditioner ran in                                       */
  int    fallbacks;          /* learned-smoother calls that fell back to SAP while the column  */
                             /* was in flight                                                   */
} ddamg_col_info;

typedef struct ddamg_stats {
  double setup_seconds;      /* wall time of the last hierarchy build                           */
  double solve_seconds;      /* wall time of the last ddamg_solve                               */
  int    outer_iters;        /* outer iterations of the last solve (max over columns)           */
  double avg_middle_iters;   /* average iterations per middle-level solve (last solve)          */
  double avg_bottom_iters;   /* average iterations per bottom-level solve (last solve)          */
  long long n_middle_solves;
  long long n_bottom_solves;
  long long n_fine_ops;      /* fine-level operator applications of the last solve              */
  long long n_sap_calls;
  int    learned_fallbacks;  /* learned-smoother calls replaced by SAP (last solve)             */
  int    col_removals;       /* compactions of the active column set (last solve)               */
  long long n_inner_iters;   /* FP32 inner FGMRES steps over all outer steps (last solve)       */
  long long n_fp16_restores; /* inner steps whose FP16 basis vector was stored again at its exact
                                norm (entry scale outside the DDAMG_KNOB_FP16_RESCALE bound)     */
  double sap_kernel_ms;      /* with DDAMG_KNOB_TIME_SAP: summed HIP-event time of the timed kernel */
                             /* launches of the last solve (else 0)                               */
  long long n_sap_kernels;   /* ... the number of those launches                                  */
  long long n_sap_kernel_tiles; /* ... and the sum of their column tiles (8 columns each)         */
  long long device_bytes;    /* device memory the context holds now (in use, or released and   */
                             /* kept for reuse by later requests of about the same size)         */
  long long device_bytes_peak; /* the largest device_bytes since the context was created        */
} ddamg_stats;

/* Fill p with the defaults of the two-level 4^4 case; callers overwrite fields. */
void ddamg_default_params(ddamg_params* p);

/* Build a context: copy the gauge field (host pointer if gauge_on_device == 0,
 * else device), set up the internal layouts and, for n_levels > 1, run the
 * adaptive setup (section 2: P and R from approximate low modes, recursively).
 * tv_init: NULL, or n_levels-1 HOST pointers to the random start vectors of
 * each level transition in canonical layout ([N][V][4][3] complex for level 0,
 * [N][Vc][2N_prev] complex for level 1); with NULL the library draws them with
 * its own counter-based generator from p->seed.  hip_stream: the stream all
 * work of this context is issued on (NULL = default stream). */
int ddamg_setup(const ddamg_params* p, const double* gauge, int gauge_on_device,
                const double* const* tv_init, void* hip_stream, ddamg_ctx** out);

/* Replace the test vectors of level transition `level` (host, canonical
 * layout as for tv_init) and rebuild P, R and every coarser operator from
 * them (the test vectors are orthonormalised per aggregate and chirality).
 * Paper section 2: the interpolation is built from a few approximate low
 * modes (test vectors), the coarse operator is the Galerkin product.  The
 * hook lets a caller (the parity tests) impose the oracle's vectors. */
int ddamg_set_test_vectors(ddamg_ctx* h, int level, const double* tv);

/* Copy out the orthonormalised test vectors (P) of a level transition, host,
 * canonical layout [N][V_l][d_l] complex with d_0 = 12. */
int ddamg_get_test_vectors(ddamg_ctx* h, int level, double* tv);

/* y_c = D_level(mu_c) x_c for n_col columns (device pointers, canonical
 * layout of that level).  Paper section 3 and Fig. 2: the operator is
 * applied to a bundle of vectors at once, each matrix entry loaded once for
 * all of them; Fig. 6 caption: D_TM = D_W + i (dmu) mu gamma5.
 * level 0 = fine operator (the paper's batched
 * operator application, each link loaded once for a tile of columns);
 * level > 0 = Galerkin coarse operator D_c(0) + i (dmu) mu_c gamma5_c.
 * precision DDAMG_FP64 or DDAMG_FP32 (FP32 uses 2-row compressed links on the
 * fine level); the canonical arrays are always FP64. */
int ddamg_apply_op(ddamg_ctx* h, int level, int precision, const double* mu, int n_col,
                   const double* x, double* y);

/* Non-degenerate twisted mass (paper section 1: the method generalised to the
 * non-degenerate doublet).  Doublet operator on psi = (psi_u, psi_d):
 *   D_ND psi = ( D(+mubar) psi_u - epsbar psi_d ,  D(-mubar) psi_d - epsbar psi_u )
 * i.e. D_W (x) 1 + i mubar gamma5 (x) tau3 - epsbar (x) tau1, with D(mu) the
 * operator above (clover term included when c_sw != 0).  n_pair doublets,
 * each with its own (mubar, epsbar) (host arrays); x, y device pointers in the
 * fine canonical layout with the two flavours of doublet i as columns 2i (u)
 * and 2i+1 (d): [pair][flavour][V][4][3]. */
int ddamg_apply_op_nd(ddamg_ctx* h, int precision, const double* mubar, const double* epsbar, int n_pair,
                      const double* x, double* y);

/* ddamg_apply_op for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, layouts and result (the same kernels), but it calls no
 * hipMalloc, hipFree or other allocating routine.  The internal-layout input
 * and output and the per-column shifts live in a device array of 64 MiB that
 * the library holds on every GPU it runs on until the process ends (its
 * address is resolved per device at the first ddamg_setup there).  A batch
 * that needs more (two internal vectors of n_col columns rounded up to whole
 * tiles of 8, plus the shifts) returns DDAMG_EINVAL with the size in
 * ddamg_last_error.  Every call on one GPU shares that array, whose contents
 * are those of the last call: calls that overlap on one GPU (several host
 * threads, or several streams) race and must be serialised by the caller. */
int ddamg_apply_op_noalloc(ddamg_ctx* h, int level, int precision, const double* mu, int n_col,
                           const double* x, double* y);

/* x_c = M_SAP(mu_c) f_c: sap_cycles red-black Schwarz cycles from x = 0 with
 * sap_mr_iters MR steps per block (section 2; fine level, device pointers).
 * precision DDAMG_FP64, DDAMG_FP32, or DDAMG_FP16: the FP32 smoother with
 * each f_c first stored in FP16 as f_c * sqrt(12 V) / 16 (V fine sites), the
 * form the inner Krylov solve uses on its FP16 basis; it needs SAP blocks of
 * 256 sites and DDAMG_KNOB_SAP_VARIANT 2 or 3 (or sap_oddeven), else
 * DDAMG_EINVAL. */
int ddamg_apply_sap(ddamg_ctx* h, int precision, const double* mu, int n_col,
                    const double* f, double* x);

/* Restriction y = P^dag x from level `level` to level+1, and prolongation
 * y = P x from level+1 to level (device pointers, canonical layouts). */
int ddamg_restrict(ddamg_ctx* h, int level, int precision, int n_col, const double* x, double* y);
int ddamg_prolong(ddamg_ctx* h, int level, int precision, int n_col, const double* x, double* y);

/* Copy out the coarse blocks of level `level` (>= 1), host, canonical layout. */
int ddamg_get_coarse_op(ddamg_ctx* h, int level, double* blocks);

/* Lattice volume and dof per site of a level (dof = 12 on level 0, 2N above). */
int ddamg_level_info(ddamg_ctx* h, int level, int* volume, int* dof, int dims[4]);

/* Solve D(mu_k) x_{r,k} = b_r for all n_rhs x n_shift columns simultaneously
 * (sections 3 and 4): FP64 flexible GMRES to relative residual p->tol,
 * preconditioned by the multigrid cycle.  b: device [n_rhs][V][4][3] complex;
 * x: device [n_rhs*n_shift][V][4][3] complex, read as initial guess when
 * use_x0 != 0, else zeros; mu: host [n_shift]; info: host, n_rhs*n_shift
 * entries or NULL.  Returns DDAMG_NOT_CONVERGED if any column misses tol. */
int ddamg_solve(ddamg_ctx* h, const double* mu, int n_shift, const double* b, int n_rhs,
                double* x, int use_x0, ddamg_col_info* info);

/* Many independent systems on the same gauge field in one simultaneous solve
 * (uneven batches): system s has n_rhs[s] right-hand sides and n_shift[s]
 * twisted masses.  mu: host, the systems' shifts one after the other
 * (sum n_shift entries); b: device, their right-hand sides one after the other
 * (sum n_rhs fields [V][4][3]); x: device, the columns of system 0
 * (rhs-major, shift fastest), then of system 1, ... (sum n_rhs*n_shift fields);
 * info: host, one entry per column, or NULL.  All columns share the hierarchy
 * and leave the solve as they converge.  Returns as ddamg_solve. */
int ddamg_solve_batch(ddamg_ctx* h, int n_sys, const int* n_rhs, const int* n_shift, const double* mu,
                      const double* b, double* x, int use_x0, ddamg_col_info* info);

/* Solve D_ND x_i = b_i for n_pair doublets (layout as ddamg_apply_op_nd; b
 * and x device pointers, x the initial guess if use_x0) to the relative
 * residual tol of each doublet (both flavours together), with FP64 flexible
 * GMRES whose Krylov vectors are the doublets (dots and norms summed over the
 * two flavour columns) and whose preconditioner is the multigrid cycle of
 * this context applied flavour by flavour with shifts +mubar and -mubar
 * (flavour diagonal; the epsbar coupling is left to the outer iteration).
 * info: 2 n_pair entries, equal within a doublet; the residuals are the
 * doublet's. */
int ddamg_solve_nd(ddamg_ctx* h, const double* mubar, const double* epsbar, int n_pair, const double* b, double* x,
                   int use_x0, ddamg_col_info* info);

/* Solve D_level(mu_c) x_c = b_c on a coarse level (level >= 1) with
 * restarted GMRES (block = 0, per column) or block GMRES (block != 0: columns
 * with equal mu form one block, section 4; block Gram-Schmidt and Cholesky QR
 * on the GPU), restart min(maxit, 63), to relative residual tol or maxit
 * (block) steps.  b, x: device, canonical layout of that level; mu: host
 * [n_col]; iters: host [n_col] or NULL.  The coarsest-level solve of the
 * multigrid cycle uses the block form when params.coarsest_block != 0. */
int ddamg_coarse_solve(ddamg_ctx* h, int level, int precision, int block, const double* mu, int n_col,
                       const double* b, double* x, double tol, int maxit, int* iters);

/* Statistics of the last setup / solve. */
int ddamg_get_stats(ddamg_ctx* h, ddamg_stats* s);

/* Time n_iter back-to-back launches of one kernel family on resident random
 * internal vectors (n_col columns, given precision) with HIP events recorded
 * on the context's stream; *sec = mean seconds per launch.  op: 0 = fine
 * stencil (level 0), 1 = SAP smoother (level 0), 2 = coarse stencil of
 * `level`, 3 = restriction from `level`, 4 = prolongation to `level`,
 * 5 = plain device copy of the multivector (reads and writes its size; a
 * kernel of known traffic for calibrating memory counters), 6 = SAP smoother
 * reading its right-hand side from FP16 storage (the form used inside the
 * inner Krylov solve; precision FP32, level 0, SAP blocks of 256 sites and
 * SAP variant 2 or 3 or sap_oddeven, else DDAMG_EINVAL). */
int ddamg_time_op(ddamg_ctx* h, int op, int level, int precision, int n_col, int n_iter, double* sec);

/* Tile-shape knobs.  DDAMG_KNOB_DSLASH_SITES_FP64: lattice sites per
 * workgroup of the FP64 fine stencil (16, 32 or 64; each workgroup stages its
 * sites x 8 columns in LDS); DDAMG_KNOB_DSLASH_SITES_FP32: the same for FP32
 * (32, 64 or 128); DDAMG_KNOB_FP32_LINKS: storage of the FP32 links read by
 * the fine stencil (0 = full 3x3 with the boundary sign folded in, 1 = 2-row
 * compressed, third row rebuilt, sign from the neighbour table).  Unknown
 * knobs or inadmissible values give DDAMG_EINVAL. */
#define DDAMG_KNOB_DSLASH_SITES_FP64 0
#define DDAMG_KNOB_DSLASH_SITES_FP32 1
#define DDAMG_KNOB_FP32_LINKS        2   /* 0: full 3x3 FP32 links; 1: 2-row compressed */
#define DDAMG_KNOB_COARSE_MFMA       3   /* FP32 coarse stencil: 1 (default) BF16 MFMA with FP32
                                            accumulation where d % 16 == 0; 0 FP32 vector kernel */
#define DDAMG_KNOB_SAP_VARIANT       4   /* FP32 SAP on 4^4 blocks: 0 (default) 2 columns per workgroup,
                                            the block's 2-row links staged in LDS; 1 2 columns, links
                                            read through L1/L2; 2 one column, 2-row links through
                                            L1/L2 (less LDS per workgroup, more workgroups per CU);
                                            3 one column, full 3x3 links through L1/L2 (no third-row
                                            rebuild in the MR steps, 1.5x the link bytes).  The
                                            odd-even form (sap_oddeven) has one kernel, 2-row links */
#define DDAMG_KNOB_DSLASH_ORDER      5   /* fine stencil scheme: 0 (default) site ranges staged in LDS,
                                            storage order; 1 the same in time-slice order; 2 / 3
                                            t-walk over columns of 4^4 blocks (psi(t-1..t+1) in
                                            registers, 4 / 8 columns per workgroup; 4^4 SAP blocks only) */
#define DDAMG_KNOB_WALK_SEGMENTS     6   /* t-walk stencil: segments of the t direction, one workgroup
                                            each (1, 2, 4 or 8; must divide Lt, else 1) */
#define DDAMG_KNOB_FP16_RESCALE      7   /* inner FGMRES with an FP16 basis: new basis vectors are
                                            stored unnormalised, at a predicted norm; when the ratio
                                            c of the true norm to the prediction leaves [1/B, B]
                                            the vector is stored again at its exact norm.  B: 1 to
                                            1024 (default 4; 1 stores every vector at its norm) */
#define DDAMG_KNOB_TIME_SAP          8   /* kernel class timed with HIP events around every launch of
                                            a solve, summed into ddamg_stats (sap_kernel_ms,
                                            n_sap_kernels, n_sap_kernel_tiles): 0 (default) off,
                                            1 the fine SAP half sweep, 2 the coarse stencil of level 1,
                                            3 the restriction 0 -> 1, 4 the prolongation 1 -> 0,
                                            5 the fine stencil */
#define DDAMG_KNOB_TIME_KERNEL       DDAMG_KNOB_TIME_SAP
#define DDAMG_KNOB_GRAM_ONE_REDUCTION 9  /* Arnoldi steps of (F)GMRES with FP32 or FP64 bases
                                            (communication-avoiding Gram-Schmidt, the outlook of
                                            sections 4 and 5: fewer global reductions per step):
                                            1 (default) one reduction per step - the dots with
                                            the basis and the new vector's own squared norm in
                                            one pass; the norm of the orthogonalised vector is
                                            predicted from them (Pythagoras), so the update pass
                                            stores it already normalised and measures its norm
                                            on the way, which gives h_{j+1,j} and decides whether
                                            a correcting rescale is needed (it is when the
                                            prediction cancelled); 0: dots, update with norm,
                                            then a normalisation pass; 2: as 1 with the
                                            correcting rescale at every step (test form) */
#define DDAMG_N_KNOBS 10
int ddamg_set_tuning(ddamg_ctx* h, int knob, int value);
int ddamg_get_tuning(ddamg_ctx* h, int knob, int* value);

/* Autotuner: for every knob, time each admissible value on resident random
 * vectors of n_col columns (HIP events on the context's stream, 10 launches
 * each), keep the fastest, and write the chosen values to values[knob]
 * (values may be NULL).  Results depend on (lattice, n_col, device) and can be
 * stored by the caller and restored with ddamg_set_tuning. */
int ddamg_autotune(ddamg_ctx* h, int n_col, int* values);

/* ---- learned smoother (gauge-covariant parallel-transport convolution net) ----
 * Two linear layers, 1 -> 2 -> 1 spinor channels:
 *   out_o(x) = sum_i sum_p W[p][o][i] (T_p in_i)(x),  p = 0 (identity), 1..4 = +mu, 5..8 = -mu,
 *   T_{+mu} f(x) = U_mu(x) f(x+mu),  T_{-mu} f(x) = U_mu(x-mu)^dag f(x-mu) (antiperiodic sign included),
 * each W[p][o][i] a complex 4x4 spin matrix (gauge covariant by construction).
 * Weights (host, double complex): layer 1 [9][2][1][4][4], layer 2 [9][1][2][4][4];
 * on the device they are stored in BF16 and used with FP32 accumulation.
 * With params.smoother = DDAMG_SMOOTHER_LEARNED the network replaces the fine
 * SAP smoother in the preconditioner: from z = 0, r = v, params.smoother_cycles
 * minimal-residual steps along p = f(r) (z += a p, r -= a D p,
 * a = <Dp, r>/<Dp, Dp>).  Whenever the network's first output does not reduce
 * the residual of every column (||v - D f(v)|| >= ||v||) SAP is used for that
 * call instead (counted in ddamg_stats.learned_fallbacks). */
int ddamg_smoother_set_weights(ddamg_ctx* h, const double* w1, const double* w2);
int ddamg_smoother_get_weights(ddamg_ctx* h, double* w1, double* w2);
/* Load / store the network weights from / to a file (host path): the 8 bytes
 * "DDAMGPTC", a little-endian int32 format version (1), then layer 1 and
 * layer 2 as little-endian double complex in the shapes above (288 + 288
 * complexes).  A missing, short, or foreign file returns DDAMG_EINVAL with
 * the reason in ddamg_last_error, and leaves the current weights unchanged. */
int ddamg_load_smoother(ddamg_ctx* h, const char* path);
int ddamg_save_smoother(ddamg_ctx* h, const char* path);
/* y = f(x), one network pass, for n_col fine vectors (device, canonical layout). */
int ddamg_smoother_apply(ddamg_ctx* h, int n_col, const double* x, double* y);
/* One layer (1 or 2), or its adjoint when adjoint != 0, on FP32 internal data:
 * in: [c_in][n_col][V][4][3] complex, out: [c_out][n_col][V][4][3] (device). */
int ddamg_ptc_layer(ddamg_ctx* h, int layer, int adjoint, int n_col, const double* in, double* out);
/* Weight gradient of one layer: g[p][o][i][s][t] = 2 sum_{x,c,col} gout_o[s][c] conj((T_p in_i)[t][c])
 * (= dL/dRe W + i dL/dIm W for gout = dL/d conj(out)); in, gout device, g host. */
int ddamg_ptc_weight_grad(ddamg_ctx* h, int layer, int n_col, const double* in, const double* gout, double* g);
/* Train the current weights with Adam on the GPU kernels from residual -> error
 * pairs that the solver iteration produces: every step draws `batch` Gaussian
 * errors e0 and applies k = step mod (sap_sweeps + 1) SAP error-propagation
 * sweeps e <- e - M_SAP D e (params.sap_cycles / sap_mr_iters); then
 * r = D(mu_c) e (mu_c cycles through mus), both scaled by 1/||r||, and Adam
 * descends the mean of ||f(r) - e||^2 / ||e||^2.  Adam's moments start from
 * zero on every call.  loss_history (host, `steps` entries) may be NULL.
 * Returns DDAMG_ESTATE if no weights were set, DDAMG_EINVAL for bad sizes. */
int ddamg_train_smoother(ddamg_ctx* h, const double* mus, int n_mu, int steps, int batch, double lr,
                         int sap_sweeps, uint64_t seed, double* loss_history);

void ddamg_destroy(ddamg_ctx* h);
const char* ddamg_strerror(int status);
/* Message of the last error raised on the calling thread ("" if none). */
const char* ddamg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DDAMG_H */
