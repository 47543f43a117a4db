/*
 * snk.h -- C ABI of the seminumerical exact-exchange (sn-K) library for MI355X (gfx950).
 *
 * The library builds the exchange matrix of hybrid Kohn-Sham DFT by the sn-K
 * factorisation of Sec. II.D of Williams-Young et al., "Distributed Memory, GPU
 * Accelerated Fock Construction for Hybrid, Gaussian Basis Density Functional
 * Theory" (arXiv 2303.14280):
 *
 *   F_{lam i}  = sum_nu P_{lam nu} Phi_{nu i}            Eq. fmat  (Phi: Eq. collocation)
 *   G_{mu i}   = w_i sum_lam A_{mu lam i} F_{lam i}      Eq. gmat  (A: Eq. 3c_grid)
 *   Kt_{mu nu} = sum_i G_{mu i} Phi_{nu i}               Eq. usym_k
 *   K          = (Kt + Kt^T) / 2                         Eq. sn_k
 *   E_x        = -1/2 tr(P K)
 *
 * evaluated per spatial batch of grid points (Sec. II.E) on one GPU.  The 3c-CP
 * integrals A are never stored: they are produced on the fly by the Obara-Saika
 * recursions of App. A (Eqs. vrr, hrr) and contracted with F in the same kernel.
 *
 * Conventions shared by every entry point
 *  - Units: bohr and hartree.
 *  - Basis: contracted Cartesian Gaussian shells, l = 0, 1, 2, 1..SNK_MAX_NPRIM
 *    primitives each (Sec. II.B, primitive form).  Components are ordered
 *    lexicographically (x,y,z; xx,xy,xz,yy,yz,zz).  `coefs` already contain the
 *    normalisation of the axis-aligned component x^l e^{-zeta r^2}; the library
 *    scales every other component to unit norm.  Basis functions are numbered
 *    shell by shell in the order given.
 *  - Matrices (P, K) are nbf x nbf, row-major, FP64.  P must be symmetric.
 *  - Ownership: the caller owns every pointer it passes.  The library copies what
 *    it needs during the call and never frees or retains caller memory.
 *  - Errors: every function returns an snk_status; no C++ exception crosses the
 *    ABI.  On SNK_E_DEVICE the HIP error text is available from snk_last_error().
 *  - Threads: a context is not thread-safe; different contexts are independent.
 */
#ifndef SNK_H
#define SNK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SNK_VERSION 1
#define SNK_MAX_L 2
#define SNK_MAX_NPRIM 8

typedef enum snk_status {
    SNK_OK = 0,
    SNK_E_ARG = 1,          /* null pointer, l > 2, nprim out of range, exponent <= 0, non-finite, weight < 0 */
    SNK_E_UNSUPPORTED = 2,  /* option not available in this library */
    SNK_E_NOMEM = 3,        /* device or host allocation failed, or the device budget is too small */
    SNK_E_DEVICE = 4,       /* HIP runtime error (text in snk_last_error) */
    SNK_E_ASYM = 5          /* validate mode: |P - P^T| > 1e-12 max|P| */
} snk_status;

typedef enum snk_precision {
    SNK_FP64 = 0,           /* every step in FP64 */
    SNK_MIXED = 1           /* with a screen and eps_basis > 0: per tile, the functions whose
                               largest |phi| over the tile's points is below 1e-3 enter both
                               dense products (Eqs. fmat, usym_k) through the FP32 matrix cores
                               (their P columns and Phi rows rounded to FP32, FP32 sums of at
                               most 1024 terms added to the FP64 products of the other
                               functions); stats->lowprec_bound is a rigorous bound on the
                               energy this moves.  Boys function, recurrences, A.F, G and K stay
                               FP64.  With a screen and eps_basis = 0: blocks whose estimated
                               energies sum to at most eps_lowprec_energy / 1e-5 per build run
                               their Boys function, recurrences and A.F contraction in FP32.
                               With SNK_FP32_GEMM: FP32 Phi/P/F and FP32 matrix-core GEMMs for
                               every function (the uniform form, outside the 1e-6 Eh budget) */
} snk_precision;

typedef enum snk_screen {
    SNK_SCREEN_NONE = 0,    /* every shell pair at every batch */
    SNK_SCREEN_BOUND = 1,   /* rigorous block bound (Sec. II.E, sn-LinK-type pair selection) */
    SNK_SCREEN_LEARNED = 2, /* MLP estimate with the rigorous bound as fallback */
    SNK_SCREEN_LINK = 3     /* the paper's pair selection (Sec. II.E, Eq. sp_set): keep (A,B) on batch
                               j when Ft_A Ft_B At_AB >= eps or max(Ft_A, Ft_B) phit_j At_AB >= eps,
                               eps = eps_skip_energy (the paper uses 1e-9).  Ft_A = max over the
                               functions mu of A of Ft_mu = sum_{nu in B_t} |P_mu,nu| Phit_nu
                               (Eq. exx_fmat_approx, mu over the whole basis, one grouped product
                               over the tiles), Phit_nu = max over the batch of sqrt(w_i)
                               |Phi_nu,i|; phit_j = max_i sqrt(w_i) sum_mu |Phi_mu,i|; At_AB = sum
                               over primitive pairs of |prefactor| max(1, |AB|)^(l_A + l_B) (a
                               global estimate of max |A_ab|).  Not an energy budget:
                               stats->skipped_bound reports the rigorous bound on the skipped
                               blocks' energy */
} snk_screen;

/* opts.flags */
#define SNK_DEVICE_PTRS 0x1u   /* P and K_out are device pointers; work is ordered on opts.stream */
#define SNK_VALIDATE    0x2u   /* check P for symmetry and finiteness (host-pointer mode) */
/* 0x4u is not a flag (rejected with SNK_E_ARG) */
#define SNK_FP32_GEMM   0x8u   /* SNK_MIXED: also store Phi, P and F in FP32 and run both dense GEMMs
                                  on the FP32 matrix cores (FP32 sums over <= 1024 terms, FP64
                                  across them); without it the mixed build's GEMMs stay FP64 */
#define SNK_OVERLAP_GROUPS 0x10u /* plain FP64 builds (no density or basis screen, FP64, at least 128
                                  batches): split the batches into two groups with their own Phi, F,
                                  G and partial-sum buffers and run them on two streams, so that one
                                  group's collocation and GEMMs, and the tail of each of its A.F
                                  launches, overlap the other's A.F work.  K is bitwise that of
                                  the sequential order (the reductions into K stay ordered); each
                                  A.F launch covers half the batches.  Ignored elsewhere; builds
                                  that return statistics run the two groups one after the other */

typedef struct snk_basis {
    int32_t nshell;
    const double* center;    /* [3*nshell] shell centres (x,y,z), host memory */
    const int32_t* l;        /* [nshell] angular momentum 0..2 */
    const int32_t* nprim;    /* [nshell] primitives per shell, 1..SNK_MAX_NPRIM */
    const int32_t* prim_off; /* [nshell] offset of the shell's first primitive in exps/coefs */
    const double* exps;      /* primitive exponents, > 0 */
    const double* coefs;     /* contraction coefficients (normalised, see above) */
} snk_basis;

typedef struct snk_grid {
    int64_t npts;                 /* number of quadrature points; 0 gives K = 0 */
    const double* xyz;            /* [3*npts] points (x,y,z interleaved), host memory */
    const int32_t* atom_of_point; /* optional [npts]: parent atom, used to form spatial batches */
} snk_grid;

typedef struct snk_stats {
    double ex;               /* E_x = -1/2 tr(P K) */
    double t_total_ms;       /* wall time of the build (host clock, includes copies in host mode) */
    double t_collocate_ms;   /* GPU time per phase, summed over batch groups (HIP events) */
    double t_fgemm_ms;
    double t_screen_ms;
    double t_afg_ms;         /* the 3c-CP A.F kernels */
    double t_kgemm_ms;
    double t_finish_ms;
    int64_t pair_points[6];      /* shell-pair x grid-point units evaluated per class ss,ps,pp,ds,dp,dd */
    int64_t pair_points_skipped; /* units dropped by screening */
    int64_t pair_points_lowprec; /* units evaluated in reduced precision */
    double skipped_bound;        /* sum of the rigorous energy bounds of the skipped units */
    int32_t n_batches;
    int32_t n_groups;
    int64_t prim_pair_points[6]; /* primitive-pair x grid-point units evaluated per class */
    double t_afg_class_ms[6];    /* GPU time of the A.F kernel of each class */
    double tile_functions;       /* |B_t|, collocated functions per tile (mean weighted by columns) */
    double tile_frows;           /* rows of F computed per tile (N_b, or |L_t| with eps_basis > 0) */
    double tile_grows;           /* rows of G in the K GEMM per tile (N_b, or |M_t| with screening and eps_basis > 0) */
    double gemm_flops_fp64;      /* flops of the two dense products (Eqs. fmat, usym_k) on the FP64 matrix cores */
    double gemm_flops_fp32;      /* ... and on the FP32 matrix cores (SNK_MIXED) */
    double lowprec_bound;        /* SNK_MIXED with basis and density screening: rigorous bound on |dE_x|
                                    from the FP32 dense products (see SNK_MIXED); 0 otherwise */
    double t_gemm_ms[4];         /* GPU time (HIP events) of the grouped dense-product launches: F on
                                    the FP64 / FP32 matrix cores, K~ on the FP64 / FP32 matrix cores */
    int64_t gemm_launches[4];    /* ... and the number of such timed launch sequences (one per group) */
    double gemm_kind_flops[4][2];/* flops of each of those four kinds on the FP64 [0] and FP32 [1] matrix
                                    cores (the fused split product of SNK_MIXED counts as "F on FP32"
                                    and has both parts) */
} snk_stats;

typedef struct snk_mlp snk_mlp;

typedef struct snk_opts {
    int32_t precision;          /* snk_precision */
    int32_t screen;             /* snk_screen */
    const snk_mlp* screener;    /* required for SNK_SCREEN_LEARNED */
    double eps_basis;           /* basis-function screening tolerance eps_B (Eq. basis_screen); 0 = off.
                                   > 0: batches are ordered spatially into tiles of at most 16;
                                   tile t collocates only the functions B_t whose sphere of
                                   radius r_cut (beyond which |phi| < eps_basis) reaches the box
                                   of the tile's points; F_t = P[:, B_t] Phi_t and only the
                                   columns B_t of K~ receive G_t Phi_t^T (Sec. II.E) */
    double eps_skip_energy;     /* total energy budget for skipped blocks (Eh); SNK_SCREEN_LINK: the
                                   per-pair thresholds eps_E = eps_K of Eq. sp_set */
    double eps_lowprec_energy;  /* SNK_MIXED: error budget of the FP32 blocks (Eh), see SNK_MIXED */
    int32_t batch_points;       /* maximum points per batch, 64..256 (default 256) */
    int32_t deterministic;      /* 1: no floating-point atomics (the default path uses none) */
    int64_t max_device_bytes;   /* workspace budget for batch groups (0 = automatic) */
    int32_t device;             /* HIP device ordinal */
    void* stream;               /* hipStream_t; NULL = the library's own stream */
    uint32_t flags;             /* SNK_DEVICE_PTRS | SNK_VALIDATE | SNK_FP32_GEMM | SNK_OVERLAP_GROUPS */
    snk_stats* stats;           /* optional output of sn_k_build */
} snk_opts;

typedef struct snk_ctx snk_ctx;

/* Fill opts with defaults: FP64, no screening, eps_basis 0, 256-point batches. */
void snk_opts_default(snk_opts* opts);

/*
 * One-shot build (Alg. 1 on one GPU): K_out = K[P] for the given basis, grid and
 * quadrature weights (`weights` [npts] host memory, >= 0).  Equivalent to
 * snk_ctx_create + snk_ctx_build + snk_ctx_destroy.  K_out is overwritten; both
 * triangles are written and the result is exactly symmetric.
 */
int sn_k_build(const snk_basis* basis, const snk_grid* grid, const double* weights,
               const double* P, double* K_out, const snk_opts* opts);

/*
 * Context API for repeated builds on one geometry (SCF reuse, Sec. II.E: the
 * batches and basis screening depend on the nuclei only).  snk_ctx_create does
 * the geometry set-up (shell-pair table, spatial batches, basis screening,
 * device workspace).  snk_ctx_build computes K for a new density; with
 * SNK_DEVICE_PTRS in the creation options P and K_out are device pointers and the
 * call is asynchronous on the context's stream, otherwise they are host pointers
 * and the call returns when K_out is written.  `stats` may be NULL.
 */
int snk_ctx_create(const snk_basis* basis, const snk_grid* grid, const double* weights,
                   const snk_opts* opts, snk_ctx** out);
int snk_ctx_build(snk_ctx* ctx, const double* P, double* K_out, snk_stats* stats);
void snk_ctx_destroy(snk_ctx* ctx);

/* Number of basis functions of a context, and its number of spatial batches. */
int snk_ctx_nbf(const snk_ctx* ctx);
int snk_ctx_nbatches(const snk_ctx* ctx);

/*
 * Batch groups and tiles.  A group (Alg. 1: the batches processed together) holds the columns
 * of one F_g and G_g; the screen and the A.F kernels run over a whole group.  A tile is a run
 * of consecutive batches of a group that shares one set B_t of collocated functions
 * (Eq. basis_screen); collocation and both GEMMs run per tile.  Without basis screening each
 * group is one tile with all N_b functions; with eps_basis > 0 tiles hold up to 16
 * spatially ordered batches.
 * snk_ctx_ngroups / snk_ctx_ntiles: their numbers.  snk_ctx_tile_info: for tile k, its
 * group, its batches [b0[k], b1[k]) in the context's batch order (see snk_ctx_point_order)
 * and nB[k] = |B_t|; host arrays of snk_ctx_ntiles entries, any may be NULL.
 * snk_ctx_tile_functions: the global indices of the tile's functions, ascending, into host
 * fn[nB[k]]; SNK_E_ARG for a bad index.
 */
int snk_ctx_ngroups(const snk_ctx* ctx);
int snk_ctx_ntiles(const snk_ctx* ctx);
int snk_ctx_tile_info(const snk_ctx* ctx, int32_t* group, int32_t* b0, int32_t* b1, int32_t* nB);
int snk_ctx_tile_functions(const snk_ctx* ctx, int32_t tile, int32_t* fn);

/*
 * Exchange-correlation potential matrix on the context's grid (Sec. II.C), the sibling of
 * sn-K that shares its collocation (Eq. collocation) and F = P Phi (Eq. fmat):
 *   rho_i = sum_mu F_mu,i Phi_mu,i,  grad rho_i = 2 sum_mu F_mu,i grad Phi_mu,i   (Eq. den_grid)
 *   E^rho_i, E^gamma_i = partial derivatives of the functional's energy per unit volume
 *     eps(rho, gamma = |grad rho|^2) at the point                               (Eq. exc_grid)
 *   Z_mu,i = w_i / 2 (E^rho_i Phi_mu,i + 4 E^gamma_i grad rho_i . grad Phi_mu,i)   (Eq. zmat)
 *   V_out = Phi Z^T + Z Phi^T (nbf x nbf, row-major, exactly symmetric)         (Eq. vxc_num)
 * and *exc_out = E_xc = sum_i w_i eps_i, *nel_out = sum_i w_i rho_i (either may be NULL).
 * The density is spin-restricted (P as for sn-K, both spins); grid points with
 * rho < 1e-12 contribute nothing.  P and V_out are host or device pointers as the context's
 * SNK_DEVICE_PTRS flag says; the call is ordered on the context's stream and returns after
 * the scalars are in host memory when exc_out or nel_out is given (host-pointer mode:
 * always synchronous).  Each call may reuse buffers of the context: calls on one context do
 * not overlap.  All arithmetic FP64; the basis and grid are the context's (its precision and
 * density screen do not apply).  With eps_basis > 0 the build runs over the context's
 * batch groups and tiles: tile t uses only its functions B_t (F_t = P[B_t, B_t] Phi_t,
 * V[B_t, B_t] += ...), dropping basis values below eps_basis as sn-K does.  SNK_E_ARG for a
 * NULL context, P or V_out, an unknown functional or (host pointers) a non-finite element of
 * P; SNK_E_ASYM with SNK_VALIDATE for an asymmetric P (host pointers); SNK_E_NOMEM when the
 * workspace (3 nbf doubles per grid point of a chunk of batches, chunks sized to
 * max_device_bytes or a quarter of free device memory; with eps_basis > 0, three buffers of
 * the largest group's tiles) does not fit.
 */
#define SNK_XC_SLATER 1   /* Dirac-Slater exchange */
#define SNK_XC_LDA    2   /* Slater exchange + Perdew-Wang 1992 correlation (zeta = 0) */
#define SNK_XC_PBE    3   /* Perdew-Burke-Ernzerhof exchange and correlation */
int snk_vxc_build(snk_ctx* ctx, const double* P, int functional, double* V_out, double* exc_out, double* nel_out);

/*
 * snk_ctx_build_kxc: snk_ctx_build and snk_vxc_build of the same density in one call.  For
 * FP64 contexts without basis screening (eps_basis = 0) and without SNK_OVERLAP_GROUPS the
 * two share each batch group's collocation Phi and F = P Phi (Eq. fmat; the paper's common
 * intermediates of the exchange and XC builds): the XC point kernel and V product run on the
 * group's Phi and F after its K product, with the XC matrix Z in the place of the exchange G
 * (no batch-group memory beyond the sn-K build's; the nbf^2 XC accumulator and its split
 * partial products sit outside opts.max_device_bytes, as K~ does).  Other contexts run the two
 * builds one after the other.  Outputs, pointer modes and error codes as for the two calls; the
 * statistics are those of sn-K, with the XC work of a shared build outside the phase timings
 * but inside t_total_ms; K_out and V_out must not overlap.
 */
int snk_ctx_build_kxc(snk_ctx* ctx, const double* P, double* K_out, int functional, double* V_out, double* exc_out,
                      double* nel_out, snk_stats* stats);

/* Diagnostics. */
const char* snk_status_string(int status);
const char* snk_last_error(const snk_ctx* ctx);   /* NULL ctx: last error of a context-free call */
int snk_version(void);

/*
 * Basis screening radius (Eq. basis_screen), host only: the radius beyond which every
 * Cartesian function of a shell of angular momentum l (contracted over nprim primitives
 * with exponents exps and coefficients coefs as in snk_basis) is below eps in magnitude;
 * -1 when the shell stays below eps everywhere.  Returns the radius in *r_out; SNK_E_ARG
 * for a NULL pointer, l outside 0..2, nprim < 1, a non-positive exponent or eps <= 0.
 */
int snk_shell_rcut(int l, const double* exps, const double* coefs, int nprim, double eps, double* r_out);

/*
 * Learned block screener (the AI form beside the plain method; no counterpart in the paper,
 * which screens with the sn-LinK estimates of Sec. II.E).  A small network,
 * 16 features -> 64 -> 64 -> 1 (SiLU), predicts log10 of the absolute energy of a
 * (shell pair, grid batch) block, sum_i w_i sum |F_a,i| |A_ab(r_i)| |F_b,i|.  With
 * SNK_SCREEN_LEARNED a block is skipped when the prediction plus the stored margin puts it
 * in the batch's skip budget and its features lie inside the stored training range; the
 * rigorous bound of SNK_SCREEN_BOUND still applies.  Parameters are FP32 device memory,
 * flattened W1[64][16], b1[64], W2[64][64], b2[64], W3[64], b3 (snk_mlp_nparams() values).
 * Features are standardised with the stored mean and std inside the kernels.
 *
 * snk_mlp_create / destroy: allocate / free a network on `device` (parameters zero).
 * snk_mlp_set_params / get_params: copy the parameters from / to host memory.
 * snk_mlp_set_normalisation: feature mean and std (host, 16 each, std > 0).
 * snk_mlp_set_range: training range of the raw features (host, 16 each) and the margin
 *   (log10 units) added to predictions by the screen.
 * snk_mlp_forward: y[n] = network(x[n][16]); device pointers; bf16 != 0 rounds weights,
 *   inputs and activations to bfloat16 and accumulates in FP32 (inference form).
 * snk_mlp_loss_grad: loss (1/n) sum_s c_s (y_s - t_s)^2, c_s = `under` if y_s < t_s else 1,
 *   and its gradient; grads is a device buffer of nparams + 1 floats (gradient, then loss).
 * snk_mlp_backward: the gradient of sum_s dy[s] y[s] with respect to the parameters for a
 *   given upstream gradient dy[n] (device), into grads (nparams + 1 floats, the last 0): the
 *   plain backward pass of the FP32 network.
 * snk_mlp_adam_step: one Adam update (beta 0.9 / 0.999, eps 1e-8) at step t >= 1.
 *
 * snk_mlp_loss_grad_noalloc: snk_mlp_loss_grad for callers that cannot allocate device memory
 *   (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).
 *   Same kernels and result; the per-workgroup partial sums live in a fixed array that each
 *   GPU holds from the first snk_mlp_create on it until the process ends (21.8 MB), so the
 *   call allocates nothing.  At most 65536 samples per call (more: SNK_E_ARG, message in
 *   snk_last_error(NULL)); the network's device must be the current device.  Every call on a
 *   GPU shares that GPU's array: calls that overlap on one GPU (different streams, threads)
 *   race and must be ordered by the caller.
 */
int snk_mlp_nparams(void);
int snk_mlp_create(int device, snk_mlp** out);
void snk_mlp_destroy(snk_mlp* mlp);
int snk_mlp_set_params(snk_mlp* mlp, const float* params);
int snk_mlp_get_params(const snk_mlp* mlp, float* params);
int snk_mlp_set_normalisation(snk_mlp* mlp, const float* mean, const float* std);
int snk_mlp_set_range(snk_mlp* mlp, const float* lo, const float* hi, float margin);
int snk_mlp_forward(const snk_mlp* mlp, const float* x, int64_t n, float* y, int bf16, void* stream);
int snk_mlp_loss_grad(snk_mlp* mlp, const float* x, const float* target, int64_t n, float under, float* grads,
                      void* stream);
int snk_mlp_loss_grad_noalloc(snk_mlp* mlp, const float* x, const float* target, int64_t n, float under,
                              float* grads, void* stream);
int snk_mlp_backward(snk_mlp* mlp, const float* x, const float* dy, int64_t n, float* grads, void* stream);
int snk_mlp_adam_step(snk_mlp* mlp, const float* grads, float lr, int t, void* stream);

/*
 * Training data for the learned screener, generated by the method itself for one density.
 * Blocks are the shell pairs that keep at least one primitive pair (snk_ctx_nblock_pairs of
 * them, ordered by class ss, ps, pp, ds, dp, dd, then by pair) on every grid batch.
 *
 * snk_ctx_block_data: for block (batch b, pair k), features[(b * npairs + k) * 16 + f]
 *   (device memory, FP32) are the 16 network inputs, and block_energy[b * npairs + k]
 *   (device memory, FP64) is the exact block magnitude
 *     t = c_AB sum_i w_i | sum_{a in A, b in B} F_a,i A_ab(r_i) F_b,i |
 *   from Eqs. fmat and 3c_grid (c_AB = 1 for A != B, 1/2 for A == B), an upper bound on the
 *   change of E_x when the block is skipped.  pair_shells (host, npairs x 2 int32) receives
 *   the shells (A, B) of each pair.  Any output may be NULL.  P follows the context's
 *   SNK_DEVICE_PTRS flag.  Feature order: l_A, l_B, log10 of the smallest exponent of A and
 *   of B, |AB|, log10 of the summed primitive-pair prefactors, log10 ||P_AB||, distance of
 *   the diffuse pair centre to the batch's bounding box, the box's half diagonal, distances
 *   of A and of B to the box, log10 of the batch weight sum, log10 of the F norms of A and B
 *   on the batch, log10 of the rigorous block bound, distance of the pair centre to the
 *   batch centroid.
 */
int64_t snk_ctx_nblock_pairs(const snk_ctx* ctx);
int snk_ctx_block_data(snk_ctx* ctx, const double* P, float* features, double* block_energy, int32_t* pair_shells);

/*
 * snk_collect_block_norms: the training samples of one density in one call: for every block
 * (batch-major, as above) its 16 features feats[k * 16 + f] and the target log10 t
 * (target[k], -40 where t <= 1e-40), both FP32 device memory of capacity `cap` blocks.
 * *n_out receives the number of blocks, nbatches * snk_ctx_nblock_pairs; SNK_E_ARG (nothing
 * written) when cap is smaller.
 */
int snk_collect_block_norms(snk_ctx* ctx, const double* P, float* feats, float* target, int64_t cap,
                            int64_t* n_out);

/* Test hooks (diagnostics, not needed to build K) are declared in snk_testing.h. */

#ifdef __cplusplus
}
#endif

#endif /* SNK_H */
