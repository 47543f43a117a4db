// Host runtime of the sn-K library: argument validation, geometry set-up (shell-pair
// table, spatial grid batches, basis screening, batch groups sized to the device
// budget), the per-density build loop of Alg. 1 on one GPU, and the C ABI of snk.h.
#include "snk.h"
#include "snk_internal.h"
#include "snk_testing.h"


#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

using namespace snk;

namespace snk {
// the learned screener's network (snk_mlp.cpp)
const MlpNorm& mlp_norm(const snk_mlp* m);
const float* mlp_params(const snk_mlp* m);
void mlp_range(const snk_mlp* m, float* lo, float* hi, float* margin, int* has_range);
int mlp_device(const snk_mlp* m);
void set_last_error(const char* msg);
}  // namespace snk

namespace {

thread_local std::string g_last_error;

const double kPi = 3.14159265358979323846;

int ncart(int l) { return (l + 1) * (l + 2) / 2; }

// A run of consecutive batches of a group that shares one set of collocated functions B_t
// (basis screening, Eq. basis_screen).  Without basis screening one tile spans its group and
// holds every function.  Collocation and both GEMMs run per tile; the screen and the A.F
// kernels run over the whole group.
struct Tile {
    int b0 = 0, b1 = 0;                 // batch range [b0, b1)
    int64_t col0 = 0;                   // first column of the tile in the group's F and G
    int64_t ncols = 0;                  // (b1 - b0) * kBatch; also the row stride of Phi_t
    int64_t phi_off = 0;                // offset of Phi_t (nB x ncols) in the Phi buffer
    std::vector<int32_t> coll_shells;   // shells collocated for this tile
    std::vector<int32_t> coll_rows;     // row of each such shell's first function in Phi_t
    std::vector<int32_t> coll_fn;       // global function index of every Phi_t row
    int32_t nB = 0;                     // rows of Phi_t
    int32_t row_off = 0;                // first row of Phi_t among the group's Phi rows
    int32_t* d_coll_shells = nullptr;
    int32_t* d_coll_rows = nullptr;
    int32_t* d_coll_fn = nullptr;
    bool all_functions = true;          // Phi_t rows == all basis functions in order
};

struct Group {
    int b0 = 0, b1 = 0;                 // batch range [b0, b1)
    int64_t ncols = 0;                  // (b1 - b0) * kBatch: columns of F_g and G_g
    std::vector<Tile> tiles;
    int64_t phi_elems = 0;              // sum of nB * ncols over the tiles
    int32_t phi_rows = 0;               // sum of nB over the tiles
    int32_t* d_fn_cat = nullptr;        // the tiles' coll_fn one after the other (eps_basis > 0)
    int32_t* d_roff = nullptr;          // [ntiles + 1] row_off of each tile, then phi_rows
};

}  // namespace

struct snk_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    snk_opts opts{};
    std::string err;

    // basis
    int nshell = 0, nbf = 0;
    std::vector<int32_t> sl, snp, spo, sfn;
    std::vector<double> scen, exps, coefs;
    std::vector<double> rcut;             // basis screening radius of each shell (eps_basis > 0)
    ShellDev* d_shells = nullptr;
    double* d_exps = nullptr;
    double* d_coefs = nullptr;

    // shell pairs
    std::vector<PairHdr> pairs;
    std::vector<PrimPair> prims;
    std::vector<int32_t> pair_a, pair_b;  // A and B shell of each pair
    PairHdr* d_pairs = nullptr;
    PrimPair* d_prims = nullptr;
    int32_t* d_runs[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int32_t* d_btasks[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int32_t nrun[6] = {0, 0, 0, 0, 0, 0};
    int64_t ntask[6] = {0, 0, 0, 0, 0, 0};        // shell pairs of a class evaluated at every batch
    int64_t task_prims[6] = {0, 0, 0, 0, 0, 0};   // surviving primitive pairs summed over those pairs
    int64_t n_prim_pairs_total = 0, n_prim_pairs_kept = 0;

    // grid
    int64_t npts = 0;
    int nbatch = 0;
    double *d_px = nullptr, *d_py = nullptr, *d_pz = nullptr, *d_pw = nullptr;
    std::vector<int32_t> batch_npts;
    std::vector<double> batch_box;        // [nbatch][6]: lower and upper corner of the batch's points
    std::vector<int64_t> col_point;       // input index of the point in each batch column, -1 = padding

    // batch groups and workspace
    std::vector<Group> groups;
    int64_t max_cols = 0;
    int64_t max_tile_cols = 0;
    int64_t max_phi = 0;                // Phi buffer elements (largest group)
    int32_t max_nB = 0;                 // largest tile function set
    int32_t tile_batches = 1;           // batches per tile (the last tile of a group may be shorter)
    int32_t max_group_tiles = 0;
    // K GEMM rows restricted per tile to the functions of kept blocks (screen + basis screening)
    bool row_restrict = false;
    int32_t* d_shell_flag = nullptr;    // [max_group_tiles][nshell]
    int32_t* d_trows = nullptr;         // [max_group_tiles][nbf]
    int32_t* d_tcount = nullptr;        // [max_group_tiles]
    int32_t* d_rinv = nullptr;          // [max_group_tiles][nbf] local row of each function per tile, -1: none
    std::vector<int32_t> tile_rows;     // rows per tile of the current group
    // F GEMM rows restricted per tile to the functions whose bound |F| >= eps_basis
    bool frow_restrict = false;
    int32_t* d_fflag = nullptr;         // [max_group_tiles][nshell]
    int32_t* d_frows = nullptr;         // [max_group_tiles][nbf]
    int32_t* d_fcount = nullptr;        // [max_group_tiles]
    double* d_mx = nullptr;             // [max_group_rows] max |Phi| of each row of a group's Phi
    int32_t max_group_rows = 0;
    int32_t* d_fn_shell = nullptr;      // [nbf] shell of each function
    std::vector<int32_t> tile_frows;    // F rows per tile of the current group
    std::vector<int32_t> bound_order;   // batches of the current group, heaviest tiles first (or empty)
    // block prefilter of the F-row test: blocks = the functions of one centre (consecutive)
    int32_t nblk = 0;
    int32_t* d_blk_fn0 = nullptr;       // [nblk + 1] first function of each block
    int32_t* d_fn_blk = nullptr;        // [nbf] block of each function
    double* d_pmax = nullptr;           // [nblk][nblk] max |P| per block pair of the current build
    int32_t* d_cand = nullptr;          // [max_group_tiles][nbf] candidate functions per tile
    int32_t* d_ncand = nullptr;         // [max_group_tiles]
    // Grouped products: problem and reduction records of the launches, staged through a host
    // mirror that is never rewritten before the stream has passed every copy out of it
    char* d_arena = nullptr;
    std::vector<char> h_arena;
    size_t arena_cur = 0;
    // Plain FP64 builds (no screen, no basis screening) run consecutive groups on two streams
    // with two buffer sets, so that one group's GEMMs overlap the other's A.F kernels; the
    // reductions into K~ stay in group order.
    bool pipe = false;
    hipStream_t pstream[2] = {};
    hipEvent_t pev_fork = nullptr, pev_k[2] = {}, pev_end[2] = {};
    double* p_Phi[2] = {};
    double* p_F[2] = {};
    double* p_G[2] = {};
    double* p_part[2] = {};
    bool zero_f_rows = false;           // write every zero row of F and G (readers of every row)
    double acc_fn = 0, acc_frows = 0, acc_grows = 0, acc_cols = 0;   // column-weighted tile sizes
    int nsplit = 1;                     // K GEMM split over points for full-width tiles
    int64_t part_elems = 0;             // capacity of the split partial-product buffer
    bool mixed = false;                 // SNK_MIXED + SNK_FP32_GEMM: FP32 Phi, P and F; FP32 matrix-core GEMMs
    // SNK_MIXED with a density screen and basis screening: per tile, the functions whose largest
    // |Phi| on the tile is below kWeakPhi enter both products through the FP32 matrix cores
    bool split = false;
    int32_t* d_perm = nullptr;          // [max_group_rows] Phi rows of each tile, strong then weak
    int32_t* d_cperm = nullptr;         // [max_group_rows] their functions
    int32_t* d_nstrong = nullptr;       // [max_group_tiles]
    std::vector<int32_t> tile_nstrong;  // strong rows per tile of the current group
    double* d_lpb = nullptr;            // [max_group_tiles * kBoundChunksPerTile + 1] bound partials, then the sum
    double acc_flops64 = 0, acc_flops32 = 0;   // dense-product flops per precision of a build
    double slot_flops[4][2] = {};              // ... per timed launch kind (F64/F32 parts)
    const double* d_P_cur = nullptr;    // density of the build in progress (device)
    // P[L_t, B_t] of every tile of a group, gathered once per build (grown on demand)
    void* d_Pc = nullptr;
    size_t pc_bytes = 0;
    // split build: the weak columns of P[L_t, B_t] and the weak rows of Phi_t in FP32
    void* d_Pw = nullptr;
    size_t pw_bytes = 0;
    void* d_Phw = nullptr;
    size_t phw_bytes = 0;
    std::vector<int64_t> tile_phw_off;  // per tile of the current group: first element of its rows in d_Phw
    float *d_Phi32 = nullptr, *d_F32 = nullptr, *d_P32 = nullptr;
    double *d_Phi = nullptr, *d_F = nullptr, *d_G = nullptr, *d_part = nullptr;
    double *d_Kt = nullptr, *d_P = nullptr, *d_K = nullptr, *d_partial = nullptr, *d_ex = nullptr;
    double* d_boys = nullptr;
    int nfinish = 256;

    hipEvent_t ev[16] = {};
    // timed builds: HIP events around the grouped product launches of the current group
    // (0: F FP64, 1: F FP32, 2: K FP64, 3: K FP32), each kind's time and launches per build
    bool timing = false;
    hipEvent_t gev[8] = {};
    bool gl[4] = {false, false, false, false};
    double gms[4] = {0, 0, 0, 0};
    int64_t gcount[4] = {0, 0, 0, 0};

    // screening (rigorous bound): static diagonal-pair lists per l, per-group work buffers
    int32_t* d_diag_sh[3] = {nullptr, nullptr, nullptr};
    int32_t* d_diag_row[3] = {nullptr, nullptr, nullptr};
    int32_t* d_diag_pb[3] = {nullptr, nullptr, nullptr};
    int32_t* d_diag_np[3] = {nullptr, nullptr, nullptr};
    int32_t n_diag[3] = {0, 0, 0};
    PrimPair32* d_dprims32 = nullptr;   // folded same-centre primitive pairs of the diagonal entries
    int32_t* d_dlist[3] = {nullptr, nullptr, nullptr};   // [max_group_tiles][n_diag[l]]
    int32_t* d_dcount = nullptr;        // [3][max_group_tiles]
    int32_t* d_shell_l = nullptr;
    int32_t* d_shell_row = nullptr;
    double* d_rowc = nullptr;           // [nbf][3] centre of the shell of each basis function
    int32_t max_group_batches = 0;
    double* d_U = nullptr;
    int32_t* d_counts = nullptr;
    int64_t* d_npairs = nullptr;
    double* d_skipped = nullptr;
    int64_t* d_run_base = nullptr;
    int64_t* d_bt_base = nullptr;
    int nlist = 6;                  // screened lists: 6 (FP64), or 12 (FP64 + FP32 per class)
    int32_t* d_bro[12] = {};
    int32_t* d_thr2 = nullptr;
    PrimPair32* d_prims32 = nullptr;
    float2* d_lun = nullptr;        // [max_group_batches][nshell] log10 U, log10 F norm
    // the paper's pair selection (SNK_SCREEN_LINK)
    double* d_fmax = nullptr;       // [max_group_batches][nshell] F-tilde of each shell per batch (sn-LinK)
    double* d_Pabs = nullptr;       // [nbf][nbf] |P| of the current build (sn-LinK)
    double* d_phimax = nullptr;     // [max_group_batches][link_ld] Phi-tilde per batch and tile row
    double* d_FtT = nullptr;        // [max_group_batches][nbf] F-tilde per batch and function
    int64_t link_ld = 0;
    bool kept_capture = false;      // testing: record the screen's kept pairs of the next group
    std::vector<int32_t> kept;      // (batch, A, B) triples
    double* d_phit = nullptr;       // [max_group_batches] max_i sqrt(w_i) sum_mu |Phi_mu,i|
    double* d_atil = nullptr;       // [npair_total] global estimate of max |A_ab|

    // learned screen: static pair features, batch geometry, per-group estimates
    const snk_mlp* mlp = nullptr;
    int64_t npair_total = 0;
    PairFeat* d_pfeat = nullptr;
    int32_t* d_pa = nullptr;        // [npair_total] shell A of each pair index
    int32_t* d_pb = nullptr;
    BatchGeo* d_geo = nullptr;      // [nbatch]
    float* d_lp = nullptr;          // [npair_total]
    float* d_est = nullptr;         // [max_group_batches][nne]: by position among the pairs with kept primitive pairs
    int32_t* d_thr = nullptr;       // [max_group_batches]
    std::vector<int32_t> ne_list;   // pair indices with kept primitive pairs, class order
    int32_t ne_class_off[7] = {0, 0, 0, 0, 0, 0, 0};
    int32_t* d_ne_list = nullptr;
    int2* d_ne_ab = nullptr;
    int32_t* d_ne_pos = nullptr;
    PairFeat* d_ne_feat = nullptr;
    int32_t* d_pool_runs[12] = {};
    int32_t* d_pool_bt[12] = {};
    int64_t cap_runs[12] = {};
    int64_t cap_bt[12] = {};

    // exchange-correlation potential (snk_vxc_build): workspace made on first use
    int64_t xc_cols = 0;                // grid columns per chunk (whole batches)
    double* d_xphi = nullptr;           // [nbf][xc_cols] Phi
    double* d_xF = nullptr;             // [nbf][xc_cols]
    double* d_xG = nullptr;             // [nbf][xc_cols] G = 2 Z
    double* d_xe = nullptr;             // [2][xc_cols] w eps, w rho per column
    double* d_xred = nullptr;           // [512] partial sums
    double* d_xsum = nullptr;           // [2] E_xc, N_el
    // sn-K and XC from one pass (snk_ctx_build_kxc): the XC point kernel and V product run on
    // each group's Phi and F right after its K product
    int kx_fn = 0;                      // functional while a combined build runs, else 0
    double* d_kxe = nullptr;            // [2][max_cols] w eps, w rho
    double* d_kxKt = nullptr;           // [nbf][nbf] unsymmetrised V
    double* d_kxred = nullptr;          // [512]
    double* d_kxsum = nullptr;          // [3] E_xc, N_el, and the finish's unused trace
    XcTile* d_kxtiles = nullptr;        // one point-kernel tile per group: every shell, from row 0
    int32_t* d_kxshells = nullptr;      // identity shell list
    int kx_nsplit = 1;
    XcTile* d_xtiles = nullptr;         // point-kernel tiles: one per chunk, or every tile of every group
    int32_t* d_xshells = nullptr;       // their shell lists, concatenated
    std::vector<int32_t> xc_gt0;        // first tile of each group in d_xtiles (basis-screened form)
    int xc_nsplit = 1;
};

namespace {

#define HIPCHECK(ctx, expr)                                                                       \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            set_err(ctx, std::string(#expr) + ": " + hipGetErrorString(e_));                      \
            return e_ == hipErrorOutOfMemory ? SNK_E_NOMEM : SNK_E_DEVICE;                        \
        }                                                                                         \
    } while (0)

void set_err(snk_ctx* ctx, const std::string& m)
{
    if (ctx) ctx->err = m;
    g_last_error = m;
}

int arg_error(snk_ctx* ctx, const std::string& m)
{
    set_err(ctx, m);
    return SNK_E_ARG;
}

bool isfin(double x) { return std::isfinite(x); }

// ---------------------------------------------------------------------------------------------
// Boys table by Gauss-Legendre quadrature of the defining integral (Eq. boys), long double.
// ---------------------------------------------------------------------------------------------
void gauss_legendre(int n, std::vector<long double>& x, std::vector<long double>& w)
{
    x.assign(n, 0.0L);
    w.assign(n, 0.0L);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        long double z = cosl(pi * (i + 0.75L) / (n + 0.5L));
        long double pp = 0.0L;
        for (int it = 0; it < 100; ++it) {
            long double p1 = 1.0L, p2 = 0.0L;
            for (int k = 1; k <= n; ++k) {
                long double p3 = p2;
                p2 = p1;
                p1 = ((2.0L * k - 1.0L) * z * p2 - (k - 1.0L) * p3) / k;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0L);
            long double dz = p1 / pp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0L / ((1.0L - z * z) * pp * pp);
    }
}

std::vector<double> make_boys_table() { return snk::boys_table_cols(kBoysCols); }

const std::vector<double>& boys_table()
{
    static const std::vector<double> t = make_boys_table();
    return t;
}

template <typename T>
int dalloc(snk_ctx* ctx, T** p, size_t n)
{
    *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void**)p, n * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        set_err(ctx, std::string("hipMalloc: ") + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? SNK_E_NOMEM : SNK_E_DEVICE;
    }
    return SNK_OK;
}

template <typename T>
int upload(snk_ctx* ctx, T** p, const std::vector<T>& v)
{
    int rc = dalloc(ctx, p, v.size());
    if (rc) return rc;
    if (!v.empty()) HIPCHECK(ctx, hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return SNK_OK;
}

// ---------------------------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------------------------
int validate_basis(snk_ctx* ctx, const snk_basis* b)
{
    if (!b) return arg_error(ctx, "basis is NULL");
    if (b->nshell < 1) return arg_error(ctx, "basis has no shells");
    if (!b->center || !b->l || !b->nprim || !b->prim_off || !b->exps || !b->coefs)
        return arg_error(ctx, "basis has a NULL array");
    for (int s = 0; s < b->nshell; ++s) {
        if (b->l[s] < 0 || b->l[s] > SNK_MAX_L) return arg_error(ctx, "shell angular momentum outside 0..2");
        if (b->nprim[s] < 1 || b->nprim[s] > SNK_MAX_NPRIM) return arg_error(ctx, "primitive count outside 1..8");
        if (b->prim_off[s] < 0) return arg_error(ctx, "negative primitive offset");
        for (int d = 0; d < 3; ++d)
            if (!isfin(b->center[3 * s + d])) return arg_error(ctx, "non-finite shell centre");
        for (int k = 0; k < b->nprim[s]; ++k) {
            const double e = b->exps[b->prim_off[s] + k], c = b->coefs[b->prim_off[s] + k];
            if (!isfin(e) || !(e > 0.0)) return arg_error(ctx, "exponent not finite and positive");
            if (!isfin(c)) return arg_error(ctx, "non-finite contraction coefficient");
        }
    }
    return SNK_OK;
}

int validate_grid(snk_ctx* ctx, const snk_grid* g, const double* w)
{
    if (!g) return arg_error(ctx, "grid is NULL");
    if (g->npts < 0) return arg_error(ctx, "negative point count");
    if (g->npts == 0) return SNK_OK;
    if (!g->xyz || !w) return arg_error(ctx, "grid points or weights are NULL");
    if (g->npts > (int64_t)1 << 40) return arg_error(ctx, "too many grid points");
    for (int64_t i = 0; i < 3 * g->npts; ++i)
        if (!isfin(g->xyz[i])) return arg_error(ctx, "non-finite grid point");
    for (int64_t i = 0; i < g->npts; ++i)
        if (!isfin(w[i]) || w[i] < 0.0) return arg_error(ctx, "weight not finite and non-negative");
    return SNK_OK;
}

// ---------------------------------------------------------------------------------------------
// set-up pieces
// ---------------------------------------------------------------------------------------------

// Shell-pair table (App. A data): unique pairs oriented l_A >= l_B, primitive pairs whose
// prefactor is below 1e-30 / max(1,|AB|)^(l_A+l_B) are dropped (their contribution is far
// below double-precision resolution of any integral of the pair).
void build_pairs(snk_ctx* c)
{
    c->pairs.clear();
    c->prims.clear();
    c->pair_a.clear();
    c->pair_b.clear();
    for (int s = 0; s < c->nshell; ++s) {
        for (int t = 0; t <= s; ++t) {
            int A = s, B = t;
            if (c->sl[t] > c->sl[s]) std::swap(A, B);
            const double* RA = &c->scen[3 * A];
            const double* RB = &c->scen[3 * B];
            const double AB[3] = {RA[0] - RB[0], RA[1] - RB[1], RA[2] - RB[2]};
            const double ab2 = AB[0] * AB[0] + AB[1] * AB[1] + AB[2] * AB[2];
            const int L = c->sl[A] + c->sl[B];
            const double grow = std::pow(std::max(1.0, std::sqrt(ab2)), L);
            PairHdr h{};
            h.prim_begin = (int32_t)c->prims.size();
            h.fa = c->sfn[A];
            h.fb = c->sfn[B];
            h.ABx = AB[0];
            h.ABy = AB[1];
            h.ABz = AB[2];
            for (int i = 0; i < c->snp[A]; ++i) {
                for (int j = 0; j < c->snp[B]; ++j) {
                    const double za = c->exps[c->spo[A] + i], zb = c->exps[c->spo[B] + j];
                    const double ca = c->coefs[c->spo[A] + i], cb = c->coefs[c->spo[B] + j];
                    const double zp = za + zb;
                    const double pref = 2.0 * kPi / zp * std::exp(-za * zb / zp * ab2) * ca * cb;
                    c->n_prim_pairs_total++;
                    if (std::fabs(pref) * grow < 1e-30) continue;
                    PrimPair q{};
                    q.zp = zp;
                    q.oo2zp = 0.5 / zp;
                    q.Px = (za * RA[0] + zb * RB[0]) / zp;
                    q.Py = (za * RA[1] + zb * RB[1]) / zp;
                    q.Pz = (za * RA[2] + zb * RB[2]) / zp;
                    q.PAx = q.Px - RA[0];
                    q.PAy = q.Py - RA[1];
                    q.PAz = q.Pz - RA[2];
                    q.pref = pref;
                    c->prims.push_back(q);
                    c->n_prim_pairs_kept++;
                }
            }
            h.nprim = (int32_t)c->prims.size() - h.prim_begin;
            c->pairs.push_back(h);
            c->pair_a.push_back(A);
            c->pair_b.push_back(B);
        }
    }
}

int class_of(int la, int lb)  // la >= lb: ss, ps, pp, ds, dp, dd
{
    static const int tab[3][3] = {{0, -1, -1}, {1, 2, -1}, {3, 4, 5}};
    return tab[la][lb];
}
const int kClassLA[6] = {0, 1, 1, 2, 2, 2};
const int kClassLB[6] = {0, 0, 1, 0, 1, 2};

// Static pair data of the learned screener's features, in pair-index order, and the list of
// pairs with kept primitive pairs in class order (the training-data layout).
int build_pair_feats(snk_ctx* c)
{
    const int64_t np = (int64_t)c->pairs.size();
    c->npair_total = np;
    std::vector<PairFeat> pf((size_t)np);
    std::vector<int32_t> pa((size_t)np), pb((size_t)np);
    std::vector<int32_t> by_class[6];
    for (int64_t p = 0; p < np; ++p) {
        const int A = c->pair_a[p], B = c->pair_b[p];
        pa[p] = A;
        pb[p] = B;
        PairFeat f{};
        double zA = 1e300, zB = 1e300;
        for (int k = 0; k < c->snp[A]; ++k) zA = std::min(zA, c->exps[c->spo[A] + k]);
        for (int k = 0; k < c->snp[B]; ++k) zB = std::min(zB, c->exps[c->spo[B] + k]);
        double ab2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double ra = c->scen[3 * A + d], rb = c->scen[3 * B + d];
            f.a[d] = (float)ra;
            f.b[d] = (float)rb;
            f.pc[d] = (float)((zA * ra + zB * rb) / (zA + zB));
            ab2 += (ra - rb) * (ra - rb);
        }
        f.la = (float)c->sl[A];
        f.lb = (float)c->sl[B];
        f.lzA = (float)std::log10(zA);
        f.lzB = (float)std::log10(zB);
        f.ab = (float)std::sqrt(ab2);
        double q = 0.0;
        const PairHdr& h = c->pairs[p];
        for (int k = 0; k < h.nprim; ++k) q += std::fabs(c->prims[h.prim_begin + k].pref);
        f.lq = q > 1e-40 ? (float)std::log10(q) : -40.0f;
        f.cab = A == B ? 0.5f : 1.0f;
        pf[p] = f;
        if (h.nprim > 0) by_class[class_of(c->sl[A], c->sl[B])].push_back((int32_t)p);
    }
    c->ne_list.clear();
    for (int k = 0; k < 6; ++k) {
        c->ne_class_off[k] = (int32_t)c->ne_list.size();
        c->ne_list.insert(c->ne_list.end(), by_class[k].begin(), by_class[k].end());
    }
    c->ne_class_off[6] = (int32_t)c->ne_list.size();
    int rc;
    if ((rc = upload(c, &c->d_pfeat, pf))) return rc;
    if ((rc = upload(c, &c->d_pa, pa))) return rc;
    if ((rc = upload(c, &c->d_pb, pb))) return rc;
    if ((rc = upload(c, &c->d_ne_list, c->ne_list))) return rc;
    std::vector<int2> ne_ab(c->ne_list.size());
    std::vector<PairFeat> ne_feat(c->ne_list.size());
    for (size_t k = 0; k < c->ne_list.size(); ++k) {
        ne_ab[k] = make_int2(pa[c->ne_list[k]], pb[c->ne_list[k]]);
        ne_feat[k] = pf[c->ne_list[k]];
    }
    if ((rc = upload(c, &c->d_ne_ab, ne_ab))) return rc;
    std::vector<int32_t> ne_pos((size_t)np, -1);
    for (size_t k = 0; k < c->ne_list.size(); ++k) ne_pos[c->ne_list[k]] = (int32_t)k;
    if ((rc = upload(c, &c->d_ne_pos, ne_pos))) return rc;
    if ((rc = upload(c, &c->d_ne_feat, ne_feat))) return rc;
    return SNK_OK;
}

// Spatial batches (Sec. II.E): per parent atom, recursive bisection on the longest
// bounding-box axis into pieces of kBatch points (one remainder piece per atom).
void split_points(const double* xyz, std::vector<int64_t>& idx, size_t lo, size_t hi,
                  std::vector<std::pair<size_t, size_t>>& out, int cap)
{
    const size_t n = hi - lo;
    if (n <= (size_t)cap) {
        if (n) out.emplace_back(lo, hi);
        return;
    }
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (size_t k = lo; k < hi; ++k)
        for (int d = 0; d < 3; ++d) {
            mn[d] = std::min(mn[d], xyz[3 * idx[k] + d]);
            mx[d] = std::max(mx[d], xyz[3 * idx[k] + d]);
        }
    int ax = 0;
    for (int d = 1; d < 3; ++d)
        if (mx[d] - mn[d] > mx[ax] - mn[ax]) ax = d;
    std::stable_sort(idx.begin() + lo, idx.begin() + hi, [&](int64_t a, int64_t b) {
        const double va = xyz[3 * a + ax], vb = xyz[3 * b + ax];
        return va < vb || (va == vb && a < b);
    });
    const size_t pieces = (n + cap - 1) / cap;
    const size_t left = ((pieces + 1) / 2) * (size_t)cap;
    split_points(xyz, idx, lo, lo + left, out, cap);
    split_points(xyz, idx, lo + left, hi, out, cap);
}

// Batches per tile when basis functions are screened: a tile's functions are those whose
// sphere reaches the tile's box, so tiles are spatially compact and small enough for the box
// to exclude distant functions.  Smaller tiles shrink B_t, L_t and M_t (the GEMMs scale with
// their products) but lower the GEMMs' rate; 16 batches (4096 columns) measured best on the
// 500- and 1000-atom clusters (8: 5% slower, 32: 10%, 128: 50%).
constexpr int kBasisTileBatches = 16;

// Plain FP64 builds of at least twice this many batches run two groups at once.
constexpr int kPipeMinBatches = 64;
// Workgroups a grouped product launch aims for (8 per compute unit): products with few output
// tiles are split over k until the launch reaches it
constexpr int64_t kGemmTarget = 2048;

// Radius beyond which every Cartesian function of a shell is below eps in magnitude, for the
// sphere test of Eq. basis_screen; -1 when the shell stays below eps everywhere.  Each
// unit-normalised component is bounded by r^l times the radial part (|x^a y^b z^c| <= r^l,
// and sqrt(3) |xy| <= sqrt(3) r^2 / 2 < r^2 for the mixed d components), so
// b(r) = r^l sum_k |c_k| exp(-zeta_k r^2) bounds the shell, and b never exceeds
// sum_k |c_k| max_r r^l exp(-zeta_k r^2) = sum_k |c_k| (l / (2 e zeta_k))^(l/2).  Every term
// of b decreases beyond r0 = sqrt(l / (2 zeta_min)); the radius is the crossing b(r) = eps
// above r0, or r0 itself when b(r0) < eps already.
double shell_rcut(int l, const double* e, const double* cf, int np, double eps)
{
    double zmin = e[0], peak = 0.0;
    for (int k = 1; k < np; ++k) zmin = std::min(zmin, e[k]);
    for (int k = 0; k < np; ++k)
        peak += std::fabs(cf[k]) * (l > 0 ? std::pow(l / (2.0 * M_E * e[k]), 0.5 * l) : 1.0);
    if (peak < eps) return -1.0;
    auto b = [&](double r) {
        double v = 0.0;
        for (int k = 0; k < np; ++k) v += std::fabs(cf[k]) * std::exp(-e[k] * r * r);
        return v * std::pow(r, l);
    };
    const double r0 = l > 0 ? std::sqrt(l / (2.0 * zmin)) : 0.0;
    if (b(r0) < eps) return r0;
    double lo = r0, hi = std::max(2.0 * r0, 1.0);
    while (b(hi) >= eps) {
        lo = hi;
        hi *= 2.0;
    }
    for (int it = 0; it < 200 && hi - lo > 1e-12 * hi; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (b(mid) >= eps) lo = mid;
        else hi = mid;
    }
    return hi;
}

int build_grid(snk_ctx* c, const snk_grid* g, const double* w)
{
    c->npts = g->npts;
    const int cap = c->opts.batch_points;
    std::vector<std::pair<size_t, size_t>> ranges;
    std::vector<int64_t> idx(g->npts);
    std::iota(idx.begin(), idx.end(), 0);
    if (g->npts > 0) {
        if (g->atom_of_point) {
            std::stable_sort(idx.begin(), idx.end(),
                             [&](int64_t a, int64_t b) { return g->atom_of_point[a] < g->atom_of_point[b]; });
            size_t lo = 0;
            while (lo < idx.size()) {
                size_t hi = lo;
                while (hi < idx.size() && g->atom_of_point[idx[hi]] == g->atom_of_point[idx[lo]]) ++hi;
                split_points(g->xyz, idx, lo, hi, ranges, cap);
                lo = hi;
            }
        } else {
            split_points(g->xyz, idx, 0, idx.size(), ranges, cap);
        }
    }
    if (c->opts.eps_basis > 0.0 && ranges.size() > (size_t)kBasisTileBatches) {
        // order the batches by recursive bisection of their centroids, so that runs of
        // kBasisTileBatches consecutive batches (the tiles) are spatially compact
        std::vector<double> cen(3 * ranges.size(), 0.0);
        for (size_t b = 0; b < ranges.size(); ++b) {
            for (size_t k = ranges[b].first; k < ranges[b].second; ++k)
                for (int d = 0; d < 3; ++d) cen[3 * b + d] += g->xyz[3 * idx[k] + d];
            for (int d = 0; d < 3; ++d) cen[3 * b + d] /= (double)(ranges[b].second - ranges[b].first);
        }
        std::vector<int64_t> order(ranges.size());
        std::iota(order.begin(), order.end(), 0);
        std::vector<std::pair<size_t, size_t>> chunks, leaves;
        split_points(cen.data(), order, 0, order.size(), chunks, kBasisTileBatches);
        // and within each tile-sized chunk down to single batches, so that shorter runs
        // (smaller groups under a tight device budget) are compact as well
        for (const auto& ch : chunks) split_points(cen.data(), order, ch.first, ch.second, leaves, 1);
        std::vector<std::pair<size_t, size_t>> sorted(ranges.size());
        for (size_t b = 0; b < order.size(); ++b) sorted[b] = ranges[order[b]];
        ranges.swap(sorted);
    }
    c->nbatch = (int)ranges.size();
    const size_t ncol = (size_t)c->nbatch * kBatch;
    std::vector<double> px(ncol), py(ncol), pz(ncol), pw(ncol, 0.0);
    c->batch_npts.assign(c->nbatch, 0);
    c->col_point.assign(ncol, -1);
    for (int b = 0; b < c->nbatch; ++b) {
        const size_t lo = ranges[b].first, hi = ranges[b].second;
        c->batch_npts[b] = (int32_t)(hi - lo);
        for (size_t k = 0; k < (size_t)kBatch; ++k) {
            const int64_t p = idx[lo + (k < hi - lo ? k : 0)];
            const size_t col = (size_t)b * kBatch + k;
            px[col] = g->xyz[3 * p];
            py[col] = g->xyz[3 * p + 1];
            pz[col] = g->xyz[3 * p + 2];
            pw[col] = k < hi - lo ? w[p] : 0.0;   // padding slots carry zero weight
            if (k < hi - lo) c->col_point[col] = p;
        }
    }
    std::vector<BatchGeo> geo(c->nbatch);
    c->batch_box.assign((size_t)c->nbatch * 6, 0.0);
    for (int b = 0; b < c->nbatch; ++b) {
        BatchGeo gb{};
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300}, ctr[3] = {0, 0, 0}, ws = 0.0;
        const int n = c->batch_npts[b];
        for (int k = 0; k < n; ++k) {
            const size_t col = (size_t)b * kBatch + k;
            const double q[3] = {px[col], py[col], pz[col]};
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], q[d]);
                hi[d] = std::max(hi[d], q[d]);
                ctr[d] += q[d];
            }
            ws += pw[col];
        }
        double hd2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            if (n == 0) lo[d] = hi[d] = 0.0;
            gb.lo[d] = (float)lo[d];
            gb.hi[d] = (float)hi[d];
            c->batch_box[6 * (size_t)b + d] = lo[d];
            c->batch_box[6 * (size_t)b + 3 + d] = hi[d];
            gb.ctr[d] = (float)(n ? ctr[d] / n : 0.0);
            hd2 += 0.25 * (hi[d] - lo[d]) * (hi[d] - lo[d]);
        }
        gb.hd = (float)std::sqrt(hd2);
        gb.lw = ws > 1e-40 ? (float)std::log10(ws) : -40.0f;
        geo[b] = gb;
    }
    int rc;
    if ((rc = upload(c, &c->d_geo, geo))) return rc;
    if ((rc = upload(c, &c->d_px, px))) return rc;
    if ((rc = upload(c, &c->d_py, py))) return rc;
    if ((rc = upload(c, &c->d_pz, pz))) return rc;
    if ((rc = upload(c, &c->d_pw, pw))) return rc;
    return SNK_OK;
}

// Batch groups (Alg. 1: as many batches as fit the device budget at once).
int build_groups(snk_ctx* c)
{
    c->groups.clear();
    // Phi, F and G columns of one batch, sized for FP64 storage in both precisions (the
    // mixed build stores Phi and F in FP32 and uses less), so that the groups, and with them
    // the basis-screened sets B_g, are the same for both
    int64_t per_batch = (int64_t)c->nbf * kBatch * 24;
    if (c->opts.screen == SNK_SCREEN_LEARNED) per_batch += (int64_t)c->ne_list.size() * (int64_t)sizeof(float);
    int64_t budget = c->opts.max_device_bytes;
    if (budget <= 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = (size_t)8 << 30;
        budget = (int64_t)(0.45 * (double)fr);
    }
    int64_t per_group = std::max<int64_t>(1, budget / per_batch);
    if (c->nbatch > 0 && per_group < 1) {
        set_err(c, "device budget smaller than one batch");
        return SNK_E_NOMEM;
    }
    const bool bscreen = c->opts.eps_basis > 0.0;
    // overlapped plain FP64 builds: at least two groups, each half of the budget (two buffer sets)
    c->pipe = (c->opts.flags & SNK_OVERLAP_GROUPS) && c->opts.screen == SNK_SCREEN_NONE && !bscreen && !c->mixed &&
              c->nbatch >= 2 * kPipeMinBatches;
    if (c->pipe) per_group = std::min<int64_t>(std::max<int64_t>(1, per_group / 2), (c->nbatch + 1) / 2);
    // with basis screening, groups are whole numbers of spatially ordered tiles
    if (bscreen && per_group > kBasisTileBatches) per_group -= per_group % kBasisTileBatches;
    const int64_t tile_batches = bscreen ? std::min<int64_t>(per_group, kBasisTileBatches) : per_group;
    c->tile_batches = (int32_t)std::max<int64_t>(1, tile_batches);
    for (int b0 = 0; b0 < c->nbatch; b0 += (int)per_group) {
        Group gr;
        gr.b0 = b0;
        gr.b1 = (int)std::min<int64_t>(c->nbatch, b0 + per_group);
        gr.ncols = (int64_t)(gr.b1 - gr.b0) * kBatch;
        for (int t0 = gr.b0; t0 < gr.b1; t0 += (int)tile_batches) {
            Tile t;
            t.b0 = t0;
            t.b1 = (int)std::min<int64_t>(gr.b1, t0 + tile_batches);
            t.col0 = (int64_t)(t0 - gr.b0) * kBatch;
            t.ncols = (int64_t)(t.b1 - t.b0) * kBatch;
            t.phi_off = gr.phi_elems;
            // B_t (Eq. basis_screen at tile level): the shells whose sphere of radius rcut
            // reaches the box of the tile's points; a superset of the union of its batches' B_j
            double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
            if (bscreen)
                for (int b = t.b0; b < t.b1; ++b)
                    for (int d = 0; d < 3; ++d) {
                        lo[d] = std::min(lo[d], c->batch_box[6 * (size_t)b + d]);
                        hi[d] = std::max(hi[d], c->batch_box[6 * (size_t)b + 3 + d]);
                    }
            int32_t row = 0;
            for (int s = 0; s < c->nshell; ++s) {
                double d2 = 0.0;
                if (bscreen) {
                    for (int d = 0; d < 3; ++d) {
                        const double x = c->scen[3 * s + d];
                        const double e = std::max(std::max(lo[d] - x, x - hi[d]), 0.0);
                        d2 += e * e;
                    }
                    if (c->rcut[s] < 0.0 || d2 > c->rcut[s] * c->rcut[s]) continue;
                }
                t.coll_shells.push_back(s);
                t.coll_rows.push_back(row);
                for (int k = 0; k < ncart(c->sl[s]); ++k) t.coll_fn.push_back(c->sfn[s] + k);
                row += ncart(c->sl[s]);
            }
            t.nB = row;
            t.all_functions = row == c->nbf;
            t.row_off = gr.phi_rows;
            gr.phi_rows += row;
            gr.phi_elems += (int64_t)t.nB * t.ncols;
            gr.tiles.push_back(std::move(t));
        }
        c->groups.push_back(std::move(gr));
    }
    c->max_cols = 0;
    c->max_tile_cols = 0;
    c->max_phi = 0;
    c->max_nB = 0;
    c->max_group_tiles = 0;
    for (auto& gr : c->groups) {
        c->max_group_tiles = std::max(c->max_group_tiles, (int32_t)gr.tiles.size());
        c->max_group_rows = std::max(c->max_group_rows, gr.phi_rows);
        c->max_cols = std::max(c->max_cols, gr.ncols);
        c->max_phi = std::max(c->max_phi, gr.phi_elems);
        for (auto& t : gr.tiles) {
            c->max_tile_cols = std::max(c->max_tile_cols, t.ncols);
            c->max_nB = std::max(c->max_nB, t.nB);
            int rc;
            if ((rc = upload(c, &t.d_coll_shells, t.coll_shells))) return rc;
            if ((rc = upload(c, &t.d_coll_rows, t.coll_rows))) return rc;
            if ((rc = upload(c, &t.d_coll_fn, t.coll_fn))) return rc;
        }
    }
    return SNK_OK;
}

int64_t pair_index(int s, int t)   // unique pair of shells s, t (stored for s >= t)
{
    if (s < t) std::swap(s, t);
    return (int64_t)s * (s + 1) / 2 + t;
}

// Runs and B tasks of every class for the unscreened build: tiles of kTileA[class]
// consecutive A shells, each sweeping all B shells (B <= A in shell order when l_A = l_B).
int build_runs(snk_ctx* c)
{
    for (int cl = 0; cl < 6; ++cl) {
        const int LA = kClassLA[cl], LB = kClassLB[cl], TA = kTileA[cl], RS = 2 + TA, BS = 2 + 2 * TA;
        std::vector<int> SA, SB;
        for (int sh = 0; sh < c->nshell; ++sh) {
            if (c->sl[sh] == LA) SA.push_back(sh);
            if (c->sl[sh] == LB) SB.push_back(sh);
        }
        std::vector<int32_t> runs, bt;
        int64_t ntask = 0, nprim = 0;
        for (size_t t0 = 0; t0 < SA.size(); t0 += TA) {
            std::vector<int32_t> rec(RS, -1);
            rec[0] = (int32_t)(bt.size() / BS);
            for (int k = 0; k < TA; ++k)
                if (t0 + k < SA.size()) rec[2 + k] = c->sfn[SA[t0 + k]];
            for (int b : SB) {
                std::vector<int32_t> brec(BS, 0);
                brec[0] = c->sfn[b];
                int mask = 0;
                for (int k = 0; k < TA && t0 + k < SA.size(); ++k) {
                    const int a = SA[t0 + k];
                    if (LA == LB && a < b) continue;
                    const int64_t p = pair_index(a, b);
                    const PairHdr& h = c->pairs[p];
                    if (h.nprim == 0) continue;   // every primitive pair negligible
                    mask |= 1 << k;
                    brec[2 + 2 * k] = h.prim_begin;
                    brec[3 + 2 * k] = h.nprim;
                    ntask += 1;
                    nprim += h.nprim;
                }
                if (!mask) continue;
                brec[1] = mask;
                bt.insert(bt.end(), brec.begin(), brec.end());
            }
            rec[1] = (int32_t)(bt.size() / BS);
            if (rec[1] > rec[0]) runs.insert(runs.end(), rec.begin(), rec.end());
        }
        c->nrun[cl] = (int32_t)(runs.size() / RS);
        c->ntask[cl] = ntask;
        c->task_prims[cl] = nprim;
        int rc = upload(c, &c->d_runs[cl], runs);
        if (rc) return rc;
        if ((rc = upload(c, &c->d_btasks[cl], bt))) return rc;
    }
    return SNK_OK;
}

// FP32 copy of the primitive-pair records (same index)
int ensure_prims32(snk_ctx* c)
{
    if (c->d_prims32) return SNK_OK;
    std::vector<PrimPair32> p32(c->prims.size());
    for (size_t k = 0; k < c->prims.size(); ++k) {
        const PrimPair& q = c->prims[k];
        p32[k] = PrimPair32{(float)q.Px, (float)q.Py, (float)q.Pz, (float)q.zp, (float)q.pref,
                            (float)q.PAx, (float)q.PAy, (float)q.PAz, (float)q.oo2zp, 0.0f};
    }
    return upload(c, &c->d_prims32, p32);
}

int setup_screening(snk_ctx* c)
{
    if (c->d_U) return SNK_OK;   // already set up
    {
        int rc = ensure_prims32(c);
        if (rc) return rc;
    }
    // Diagonal entries: the same-shell pair (A, A) of every shell, with its primitive pairs
    // folded by symmetry ((i, j) and (j, i) give the same integral: one record of twice the
    // prefactor), centred exactly on R_A.
    std::vector<PrimPair32> dp;
    for (int l = 0; l < 3; ++l) {
        std::vector<int32_t> sh, row, pb, np;
        for (int s = 0; s < c->nshell; ++s) {
            if (c->sl[s] != l) continue;
            const double* RA = &c->scen[3 * s];
            sh.push_back(s);
            row.push_back(c->sfn[s]);
            pb.push_back((int32_t)dp.size());
            for (int i = 0; i < c->snp[s]; ++i)
                for (int j = i; j < c->snp[s]; ++j) {
                    const double za = c->exps[c->spo[s] + i], zb = c->exps[c->spo[s] + j];
                    const double zp = za + zb;
                    const double pref = (i == j ? 1.0 : 2.0) * 2.0 * kPi / zp * c->coefs[c->spo[s] + i] *
                                        c->coefs[c->spo[s] + j];
                    if (std::fabs(pref) < 1e-30) continue;   // the pair table's cutoff at R_AB = 0
                    dp.push_back(PrimPair32{(float)RA[0], (float)RA[1], (float)RA[2], (float)zp, (float)pref, 0.0f,
                                            0.0f, 0.0f, (float)(0.5 / zp), 0.0f});
                }
            np.push_back((int32_t)dp.size() - pb.back());
        }
        c->n_diag[l] = (int32_t)sh.size();
        int rc;
        if ((rc = upload(c, &c->d_diag_sh[l], sh))) return rc;
        if ((rc = upload(c, &c->d_diag_row[l], row))) return rc;
        if ((rc = upload(c, &c->d_diag_pb[l], pb))) return rc;
        if ((rc = upload(c, &c->d_diag_np[l], np))) return rc;
    }
    if (dp.empty()) dp.push_back(PrimPair32{});
    {
        int rc = upload(c, &c->d_dprims32, dp);
        if (rc) return rc;
    }
    int rc;
    int32_t mb = 0;
    for (const auto& g : c->groups) mb = std::max(mb, g.b1 - g.b0);
    c->max_group_batches = mb;
    if ((rc = dalloc(c, &c->d_U, (size_t)mb * c->nshell))) return rc;
    if ((rc = dalloc(c, &c->d_lun, (size_t)mb * c->nshell))) return rc;
    if ((rc = dalloc(c, &c->d_lp, c->ne_list.size()))) return rc;
    if (c->opts.screen == SNK_SCREEN_LEARNED) {
        if ((rc = dalloc(c, &c->d_est, std::max<size_t>(1, (size_t)mb * c->ne_list.size())))) return rc;
        if ((rc = dalloc(c, &c->d_thr, (size_t)mb))) return rc;
        if ((rc = dalloc(c, &c->d_thr2, (size_t)mb))) return rc;
    }
    if (c->opts.screen == SNK_SCREEN_LINK) {
        if ((rc = dalloc(c, &c->d_fmax, (size_t)mb * c->nshell))) return rc;
        int32_t maxB = 1;
        for (const auto& g : c->groups)
            for (const Tile& t : g.tiles) maxB = std::max(maxB, t.nB);
        c->link_ld = (maxB + 3) & ~3;
        if ((rc = dalloc(c, &c->d_Pabs, (size_t)c->nbf * c->nbf))) return rc;
        if ((rc = dalloc(c, &c->d_phimax, (size_t)mb * c->link_ld))) return rc;
        if ((rc = dalloc(c, &c->d_FtT, (size_t)mb * c->nbf))) return rc;
        if ((rc = dalloc(c, &c->d_phit, (size_t)mb))) return rc;
        // At_AB = sum over primitive pairs of |prefactor| max(1, |AB|)^(l_A + l_B)
        std::vector<double> at(c->npair_total, 0.0);
        for (int a = 0; a < c->nshell; ++a)
            for (int b = 0; b <= a; ++b) {
                const int64_t p = pair_index(a, b);
                const PairHdr& h = c->pairs[p];
                const double ab = std::sqrt(h.ABx * h.ABx + h.ABy * h.ABy + h.ABz * h.ABz);
                double v = 0.0;
                for (int k = 0; k < h.nprim; ++k) v += std::fabs(c->prims[h.prim_begin + k].pref);
                at[p] = v * std::pow(std::max(1.0, ab), c->sl[a] + c->sl[b]);
            }
        if ((rc = upload(c, &c->d_atil, at))) return rc;
    }
    if ((rc = dalloc(c, &c->d_counts, (size_t)mb * 2 * c->nlist))) return rc;
    if ((rc = dalloc(c, &c->d_npairs, (size_t)mb * c->nlist))) return rc;
    if ((rc = dalloc(c, &c->d_skipped, (size_t)mb))) return rc;
    if ((rc = dalloc(c, &c->d_run_base, (size_t)c->nlist * (mb + 1)))) return rc;
    if ((rc = dalloc(c, &c->d_bt_base, (size_t)c->nlist * (mb + 1)))) return rc;
    for (int k = 0; k < c->nlist; ++k)
        if ((rc = dalloc(c, &c->d_bro[k], (size_t)mb + 1))) return rc;
    return SNK_OK;
}

// grow the run / B-task pools of class k to hold nrun runs and nbt B tasks
int ensure_pools(snk_ctx* c, int k, int64_t nrun, int64_t nbt)
{
    const int TA = kListTile(k);
    if (nrun > c->cap_runs[k]) {
        (void)hipFree(c->d_pool_runs[k]);
        const int64_t cap = std::max<int64_t>(nrun + nrun / 4, 1024);
        int rc = dalloc(c, &c->d_pool_runs[k], (size_t)cap * (2 + TA));
        if (rc) return rc;
        c->cap_runs[k] = cap;
    }
    if (nbt > c->cap_bt[k]) {
        (void)hipFree(c->d_pool_bt[k]);
        const int64_t cap = std::max<int64_t>(nbt + nbt / 4, 4096);
        int rc = dalloc(c, &c->d_pool_bt[k], (size_t)cap * (2 + 2 * TA));
        if (rc) return rc;
        c->cap_bt[k] = cap;
    }
    return SNK_OK;
}

void free_ctx(snk_ctx* c)
{
    if (!c) return;
    (void)hipFree(c->d_shells);
    (void)hipFree(c->d_exps);
    (void)hipFree(c->d_coefs);
    (void)hipFree(c->d_pairs);
    (void)hipFree(c->d_prims);
    for (int k = 0; k < 6; ++k) {
        (void)hipFree(c->d_runs[k]);
        (void)hipFree(c->d_btasks[k]);
    }
    (void)hipFree(c->d_px);
    (void)hipFree(c->d_py);
    (void)hipFree(c->d_pz);
    (void)hipFree(c->d_pw);
    for (auto& g : c->groups) {
        (void)hipFree(g.d_fn_cat);
        (void)hipFree(g.d_roff);
        for (auto& t : g.tiles) {
            (void)hipFree(t.d_coll_shells);
            (void)hipFree(t.d_coll_rows);
            (void)hipFree(t.d_coll_fn);
        }
    }
    (void)hipFree(c->d_Phi32);
    (void)hipFree(c->d_F32);
    (void)hipFree(c->d_P32);
    (void)hipFree(c->d_shell_flag);
    (void)hipFree(c->d_trows);
    (void)hipFree(c->d_tcount);
    (void)hipFree(c->d_rinv);
    (void)hipFree(c->d_arena);
    (void)hipFree(c->d_perm);
    (void)hipFree(c->d_cperm);
    (void)hipFree(c->d_nstrong);
    (void)hipFree(c->d_lpb);
    (void)hipFree(c->d_Pc);
    (void)hipFree(c->d_Pw);
    (void)hipFree(c->d_Phw);
    for (int k = 0; k < 2; ++k) {
        if (c->pstream[k]) (void)hipStreamDestroy(c->pstream[k]);
        if (c->pev_k[k]) (void)hipEventDestroy(c->pev_k[k]);
        if (c->pev_end[k]) (void)hipEventDestroy(c->pev_end[k]);
    }
    if (c->pev_fork) (void)hipEventDestroy(c->pev_fork);
    // the second buffer set (the first is the context's own)
    (void)hipFree(c->p_Phi[1]);
    (void)hipFree(c->p_F[1]);
    (void)hipFree(c->p_G[1]);
    (void)hipFree(c->p_part[1]);
    (void)hipFree(c->d_fflag);
    (void)hipFree(c->d_frows);
    (void)hipFree(c->d_fcount);
    (void)hipFree(c->d_mx);
    (void)hipFree(c->d_fn_shell);
    (void)hipFree(c->d_blk_fn0);
    (void)hipFree(c->d_fn_blk);
    (void)hipFree(c->d_pmax);
    (void)hipFree(c->d_cand);
    (void)hipFree(c->d_ncand);
    (void)hipFree(c->d_Phi);
    (void)hipFree(c->d_F);
    (void)hipFree(c->d_G);
    (void)hipFree(c->d_part);
    (void)hipFree(c->d_Kt);
    (void)hipFree(c->d_P);
    (void)hipFree(c->d_K);
    (void)hipFree(c->d_xphi);
    (void)hipFree(c->d_xF);
    (void)hipFree(c->d_xG);
    (void)hipFree(c->d_xe);
    (void)hipFree(c->d_xred);
    (void)hipFree(c->d_xsum);
    (void)hipFree(c->d_xtiles);
    (void)hipFree(c->d_xshells);
    for (double* p : {c->d_kxe, c->d_kxKt, c->d_kxred, c->d_kxsum}) (void)hipFree(p);
    (void)hipFree(c->d_kxtiles);
    (void)hipFree(c->d_kxshells);
    (void)hipFree(c->d_partial);
    (void)hipFree(c->d_ex);
    (void)hipFree(c->d_boys);
    for (auto& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : c->gev)
        if (e) (void)hipEventDestroy(e);
    for (int l = 0; l < 3; ++l) {
        (void)hipFree(c->d_diag_sh[l]);
        (void)hipFree(c->d_diag_row[l]);
        (void)hipFree(c->d_diag_pb[l]);
        (void)hipFree(c->d_diag_np[l]);
        (void)hipFree(c->d_dlist[l]);
    }
    (void)hipFree(c->d_dprims32);
    (void)hipFree(c->d_dcount);
    (void)hipFree(c->d_shell_l);
    (void)hipFree(c->d_shell_row);
    (void)hipFree(c->d_rowc);
    (void)hipFree(c->d_U);
    (void)hipFree(c->d_lun);
    (void)hipFree(c->d_fmax);
    (void)hipFree(c->d_Pabs);
    (void)hipFree(c->d_phimax);
    (void)hipFree(c->d_FtT);
    (void)hipFree(c->d_phit);
    (void)hipFree(c->d_atil);
    (void)hipFree(c->d_pfeat);
    (void)hipFree(c->d_pa);
    (void)hipFree(c->d_pb);
    (void)hipFree(c->d_geo);
    (void)hipFree(c->d_lp);
    (void)hipFree(c->d_est);
    (void)hipFree(c->d_thr);
    (void)hipFree(c->d_thr2);
    (void)hipFree(c->d_prims32);
    (void)hipFree(c->d_ne_list);
    (void)hipFree(c->d_ne_ab);
    (void)hipFree(c->d_ne_pos);
    (void)hipFree(c->d_ne_feat);
    (void)hipFree(c->d_counts);
    (void)hipFree(c->d_npairs);
    (void)hipFree(c->d_skipped);
    (void)hipFree(c->d_run_base);
    (void)hipFree(c->d_bt_base);
    for (int k = 0; k < 12; ++k) {
        (void)hipFree(c->d_bro[k]);
        (void)hipFree(c->d_pool_runs[k]);
        (void)hipFree(c->d_pool_bt[k]);
    }
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

double ev_ms(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return (double)ms;
}

}  // namespace

// =============================================================================================
// C ABI
// =============================================================================================
extern "C" {

void snk_opts_default(snk_opts* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = SNK_FP64;
    o->screen = SNK_SCREEN_NONE;
    o->eps_basis = 0.0;
    o->eps_skip_energy = 5e-7;
    o->eps_lowprec_energy = 5e-7;
    o->batch_points = kBatch;
    o->deterministic = 1;
}

int snk_version(void) { return SNK_VERSION; }

const char* snk_status_string(int s)
{
    switch (s) {
        case SNK_OK: return "ok";
        case SNK_E_ARG: return "invalid argument";
        case SNK_E_UNSUPPORTED: return "unsupported option";
        case SNK_E_NOMEM: return "out of memory";
        case SNK_E_DEVICE: return "device error";
        case SNK_E_ASYM: return "density matrix not symmetric";
        default: return "unknown status";
    }
}

const char* snk_last_error(const snk_ctx* ctx) { return ctx ? ctx->err.c_str() : g_last_error.c_str(); }

int snk_ctx_nbf(const snk_ctx* ctx) { return ctx ? ctx->nbf : 0; }
int snk_ctx_nbatches(const snk_ctx* ctx) { return ctx ? ctx->nbatch : 0; }

int snk_ctx_create(const snk_basis* basis, const snk_grid* grid, const double* weights, const snk_opts* opts,
                   snk_ctx** out)
{
    if (!out) return arg_error(nullptr, "output context pointer is NULL");
    *out = nullptr;
    snk_opts o;
    snk_opts_default(&o);
    if (opts) o = *opts;
    if (o.batch_points == 0) o.batch_points = kBatch;
    int rc = validate_basis(nullptr, basis);
    if (rc) return rc;
    if ((rc = validate_grid(nullptr, grid, weights))) return rc;
    if (o.precision != SNK_FP64 && o.precision != SNK_MIXED) return arg_error(nullptr, "unknown precision");
    if (o.screen < SNK_SCREEN_NONE || o.screen > SNK_SCREEN_LINK) return arg_error(nullptr, "unknown screen mode");
    if (o.batch_points < 1 || o.batch_points > kBatch) return arg_error(nullptr, "batch_points outside 1..256");
    if (!isfin(o.eps_basis) || o.eps_basis < 0.0) return arg_error(nullptr, "eps_basis must be >= 0");
    if (o.screen != SNK_SCREEN_NONE && (!isfin(o.eps_skip_energy) || o.eps_skip_energy < 0.0))
        return arg_error(nullptr, "eps_skip_energy must be finite and >= 0");
    if (o.flags & ~(uint32_t)(SNK_DEVICE_PTRS | SNK_VALIDATE | SNK_FP32_GEMM | SNK_OVERLAP_GROUPS))
        return arg_error(nullptr, "unknown flag");
    if (o.screen == SNK_SCREEN_LEARNED) {
        if (!o.screener) return arg_error(nullptr, "SNK_SCREEN_LEARNED needs a screener network");
        float lo[16], hi[16], margin;
        int has_range = 0;
        mlp_range(o.screener, lo, hi, &margin, &has_range);
        if (!has_range) return arg_error(nullptr, "screener network has no training range set");
        if (mlp_device(o.screener) != o.device) return arg_error(nullptr, "screener network is on another device");
    }

    snk_ctx* c = new (std::nothrow) snk_ctx();
    if (!c) return SNK_E_NOMEM;
    c->opts = o;
    c->device = o.device;
    c->mixed = o.precision == SNK_MIXED && (o.flags & SNK_FP32_GEMM);
    {
        hipError_t e = hipSetDevice(c->device);
        if (e != hipSuccess) {
            set_err(c, std::string("hipSetDevice: ") + hipGetErrorString(e));
            g_last_error = c->err;
            free_ctx(c);
            return SNK_E_DEVICE;
        }
    }
#define CREATE_CHECK(x)       \
    do {                      \
        int rc_ = (x);        \
        if (rc_) {            \
            g_last_error = c->err; \
            free_ctx(c);      \
            return rc_;       \
        }                     \
    } while (0)

    if (o.stream) {
        c->stream = (hipStream_t)o.stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            set_err(c, std::string("hipStreamCreate: ") + hipGetErrorString(e));
            g_last_error = c->err;
            free_ctx(c);
            return SNK_E_DEVICE;
        }
        c->own_stream = true;
    }
    for (auto& e : c->ev) CREATE_CHECK(hipEventCreate(&e) == hipSuccess ? SNK_OK : SNK_E_DEVICE);
    for (auto& e : c->gev) CREATE_CHECK(hipEventCreate(&e) == hipSuccess ? SNK_OK : SNK_E_DEVICE);

    // basis
    c->nshell = basis->nshell;
    c->sl.assign(basis->l, basis->l + c->nshell);
    c->snp.assign(basis->nprim, basis->nprim + c->nshell);
    c->spo.resize(c->nshell);
    c->scen.assign(basis->center, basis->center + 3 * c->nshell);
    c->sfn.resize(c->nshell);
    std::vector<ShellDev> sh(c->nshell);
    int fn = 0;
    for (int s = 0; s < c->nshell; ++s) {
        c->sfn[s] = fn;
        fn += ncart(c->sl[s]);
        c->spo[s] = (int32_t)c->exps.size();
        for (int k = 0; k < c->snp[s]; ++k) {
            c->exps.push_back(basis->exps[basis->prim_off[s] + k]);
            c->coefs.push_back(basis->coefs[basis->prim_off[s] + k]);
        }
        sh[s] = ShellDev{c->scen[3 * s], c->scen[3 * s + 1], c->scen[3 * s + 2], c->sl[s], c->snp[s], c->spo[s], 0};
    }
    c->nbf = fn;
    if (o.eps_basis > 0.0) {
        c->rcut.resize(c->nshell);
        for (int s = 0; s < c->nshell; ++s)
            c->rcut[s] = shell_rcut(c->sl[s], &c->exps[c->spo[s]], &c->coefs[c->spo[s]], c->snp[s], o.eps_basis);
    }
    CREATE_CHECK(upload(c, &c->d_shells, sh));
    CREATE_CHECK(upload(c, &c->d_exps, c->exps));
    CREATE_CHECK(upload(c, &c->d_coefs, c->coefs));

    build_pairs(c);
    CREATE_CHECK(upload(c, &c->d_pairs, c->pairs));
    CREATE_CHECK(upload(c, &c->d_prims, c->prims));
    // the mixed build evaluates the screen's small blocks in FP32
    // FP32 A.F lists in the mixed build with a density screen, except where the dense products
    // split by function magnitude (basis screening as well): there the screens skip nearly all
    // the blocks the FP32 lists would take, and the extra lists cost more than they save
    const bool split_products = o.precision == SNK_MIXED && !(o.flags & SNK_FP32_GEMM) &&
                                o.screen != SNK_SCREEN_NONE && o.eps_basis > 0.0;
    c->nlist = (o.precision == SNK_MIXED && o.screen != SNK_SCREEN_NONE && !split_products) ? 12 : 6;
    // FP32 records: the mixed build's FP32 blocks and the screen's diagonal bounds
    if (c->nlist == 12 || o.screen != SNK_SCREEN_NONE) CREATE_CHECK(ensure_prims32(c));
    CREATE_CHECK(build_pair_feats(c));
    c->mlp = o.screen == SNK_SCREEN_LEARNED ? o.screener : nullptr;
    CREATE_CHECK(build_runs(c));
    CREATE_CHECK(build_grid(c, grid, weights));
    CREATE_CHECK(build_groups(c));
    CREATE_CHECK(upload(c, &c->d_boys, boys_table()));
    // angular momentum and first function of every shell (screens and tile row lists)
    CREATE_CHECK(upload(c, &c->d_shell_l, c->sl));
    CREATE_CHECK(upload(c, &c->d_shell_row, c->sfn));
    {
        // the A.F kernels form R_A - R_B from these (the pair table's own difference)
        std::vector<double> rowc(3 * (size_t)c->nbf, 0.0);
        for (int sh = 0; sh < c->nshell; ++sh)
            for (int k = 0; k < ncart(c->sl[sh]); ++k)
                for (int d = 0; d < 3; ++d) rowc[3 * (size_t)(c->sfn[sh] + k) + d] = c->scen[3 * sh + d];
        CREATE_CHECK(upload(c, &c->d_rowc, rowc));
    }

    // workspace
    const int64_t nbf = c->nbf;
    {
        const int64_t tiles = ((nbf + 127) / 128) * ((c->max_nB + 127) / 128);
        int ns = (int)std::max<int64_t>(1, (kGemmTarget + tiles - 1) / std::max<int64_t>(1, tiles));
        ns = (int)std::min<int64_t>(ns, std::max<int64_t>(1, c->max_tile_cols / kBatch));
        c->nsplit = std::max(1, std::min(ns, 256));
    }
    if (c->mixed) {
        CREATE_CHECK(dalloc(c, &c->d_Phi32, (size_t)std::max<int64_t>(1, c->max_phi)));
        CREATE_CHECK(dalloc(c, &c->d_F32, (size_t)nbf * c->max_cols));
        CREATE_CHECK(dalloc(c, &c->d_P32, (size_t)nbf * nbf));
    } else {
        CREATE_CHECK(dalloc(c, &c->d_Phi, (size_t)std::max<int64_t>(1, c->max_phi)));
        CREATE_CHECK(dalloc(c, &c->d_F, (size_t)nbf * c->max_cols));
    }
    CREATE_CHECK(dalloc(c, &c->d_G, (size_t)nbf * c->max_cols));
    // partial products of the K GEMM: fixed size for full-width tiles (also the overlapped
    // build's second set); grown on demand when the rows are restricted per tile
    c->part_elems = std::max<int64_t>(1, (int64_t)c->nsplit * nbf * c->max_nB);
    CREATE_CHECK(dalloc(c, &c->d_part, (size_t)c->part_elems));
    CREATE_CHECK(dalloc(c, &c->d_Kt, (size_t)nbf * nbf));
    CREATE_CHECK(dalloc(c, &c->d_P, (size_t)nbf * nbf));
    CREATE_CHECK(dalloc(c, &c->d_K, (size_t)nbf * nbf));
    CREATE_CHECK(dalloc(c, &c->d_partial, (size_t)c->nfinish));
    CREATE_CHECK(dalloc(c, &c->d_ex, 1));
    if (o.screen != SNK_SCREEN_NONE) CREATE_CHECK(setup_screening(c));
    c->row_restrict = o.screen != SNK_SCREEN_NONE && o.eps_basis > 0.0 && !c->groups.empty();
    c->frow_restrict = o.eps_basis > 0.0 && !c->groups.empty();
    if (c->row_restrict) {
        CREATE_CHECK(dalloc(c, &c->d_shell_flag, (size_t)c->max_group_tiles * c->nshell));
        CREATE_CHECK(dalloc(c, &c->d_trows, (size_t)c->max_group_tiles * nbf));
        CREATE_CHECK(dalloc(c, &c->d_tcount, (size_t)c->max_group_tiles));
    }
    // per group: the tiles' function lists one after the other and their row offsets
    for (auto& g : c->groups) {
        std::vector<int32_t> cat, roff;
        for (const auto& t : g.tiles) {
            roff.push_back((int32_t)cat.size());
            cat.insert(cat.end(), t.coll_fn.begin(), t.coll_fn.end());
        }
        roff.push_back((int32_t)cat.size());
        if (cat.empty()) cat.push_back(0);
        CREATE_CHECK(upload(c, &g.d_fn_cat, cat));
        CREATE_CHECK(upload(c, &g.d_roff, roff));
    }
    if (c->frow_restrict) {
        CREATE_CHECK(dalloc(c, &c->d_fflag, (size_t)c->max_group_tiles * c->nshell));
        CREATE_CHECK(dalloc(c, &c->d_frows, (size_t)c->max_group_tiles * nbf));
        CREATE_CHECK(dalloc(c, &c->d_fcount, (size_t)c->max_group_tiles));
        CREATE_CHECK(dalloc(c, &c->d_mx, (size_t)std::max<int32_t>(1, c->max_group_rows)));
        std::vector<int32_t> fs(nbf);
        for (int sh = 0; sh < c->nshell; ++sh)
            for (int k = 0; k < ncart(c->sl[sh]); ++k) fs[c->sfn[sh] + k] = sh;
        CREATE_CHECK(upload(c, &c->d_fn_shell, fs));
        // Centre blocks for the prefilter of the F-row test: runs of consecutive shells on one
        // centre, whose functions are consecutive.  Left out (every function tested) when the
        // functions do not follow the shell order or the block-pair table would pass 256 MiB.
        std::vector<int32_t> fn0, fblk(nbf);
        bool ok = true;
        for (int sh = 0, f = 0; sh < c->nshell && ok; ++sh) {
            ok = c->sfn[sh] == f;
            if (sh == 0 || c->scen[3 * sh] != c->scen[3 * sh - 3] || c->scen[3 * sh + 1] != c->scen[3 * sh - 2] ||
                c->scen[3 * sh + 2] != c->scen[3 * sh - 1])
                fn0.push_back(f);
            for (int k = 0; k < ncart(c->sl[sh]); ++k) fblk[f + k] = (int32_t)fn0.size() - 1;
            f += ncart(c->sl[sh]);
        }
        fn0.push_back((int32_t)nbf);
        const int64_t nblk = (int64_t)fn0.size() - 1;
        if (ok && nblk > 0 && nblk * nblk * (int64_t)sizeof(double) <= ((int64_t)256 << 20)) {
            c->nblk = (int32_t)nblk;
            CREATE_CHECK(upload(c, &c->d_blk_fn0, fn0));
            CREATE_CHECK(upload(c, &c->d_fn_blk, fblk));
            CREATE_CHECK(dalloc(c, &c->d_pmax, (size_t)(nblk * nblk)));
            CREATE_CHECK(dalloc(c, &c->d_cand, (size_t)c->max_group_tiles * nbf));
            CREATE_CHECK(dalloc(c, &c->d_ncand, (size_t)std::max<int32_t>(1, c->max_group_tiles)));
        }
    }
    if (c->row_restrict || c->frow_restrict)
        CREATE_CHECK(dalloc(c, &c->d_rinv, (size_t)std::max<int32_t>(1, c->max_group_tiles) * nbf));
    c->split = o.precision == SNK_MIXED && !c->mixed && c->row_restrict && c->frow_restrict;
    if (c->split) {
        CREATE_CHECK(dalloc(c, &c->d_perm, (size_t)std::max<int32_t>(1, c->max_group_rows)));
        CREATE_CHECK(dalloc(c, &c->d_cperm, (size_t)std::max<int32_t>(1, c->max_group_rows)));
        CREATE_CHECK(dalloc(c, &c->d_nstrong, (size_t)std::max<int32_t>(1, c->max_group_tiles)));
        CREATE_CHECK(dalloc(c, &c->d_lpb, (size_t)std::max<int32_t>(1, c->max_group_tiles) * kBoundChunksPerTile + 1));
    }
    if (c->pipe) {
        c->p_Phi[0] = c->d_Phi;
        c->p_F[0] = c->d_F;
        c->p_G[0] = c->d_G;
        c->p_part[0] = c->d_part;
        CREATE_CHECK(dalloc(c, &c->p_Phi[1], (size_t)std::max<int64_t>(1, c->max_phi)));
        CREATE_CHECK(dalloc(c, &c->p_F[1], (size_t)nbf * c->max_cols));
        CREATE_CHECK(dalloc(c, &c->p_G[1], (size_t)nbf * c->max_cols));
        CREATE_CHECK(dalloc(c, &c->p_part[1], (size_t)c->part_elems));
        CREATE_CHECK(hipEventCreateWithFlags(&c->pev_fork, hipEventDisableTiming) == hipSuccess ? SNK_OK : SNK_E_DEVICE);
        for (int k = 0; k < 2; ++k) {
            CREATE_CHECK(hipStreamCreateWithFlags(&c->pstream[k], hipStreamNonBlocking) == hipSuccess ? SNK_OK
                                                                                                       : SNK_E_DEVICE);
            CREATE_CHECK(hipEventCreateWithFlags(&c->pev_k[k], hipEventDisableTiming) == hipSuccess ? SNK_OK
                                                                                                    : SNK_E_DEVICE);
            CREATE_CHECK(hipEventCreateWithFlags(&c->pev_end[k], hipEventDisableTiming) == hipSuccess ? SNK_OK
                                                                                                      : SNK_E_DEVICE);
        }
    }
#undef CREATE_CHECK
    *out = c;
    return SNK_OK;
}

void snk_ctx_destroy(snk_ctx* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    free_ctx(ctx);
}

}  // extern "C"

namespace {

struct GroupStats {
    int64_t pp[6] = {0, 0, 0, 0, 0, 0};    // shell-pair x point units evaluated
    int64_t ppp[6] = {0, 0, 0, 0, 0, 0};   // primitive-pair x point units evaluated
    int64_t cand = 0;                       // units before density screening
    int64_t low = 0;                        // units evaluated in FP32
    double skipped = 0.0;                   // bound on the energy of the skipped blocks
};

int group_fgemm(snk_ctx* c, const Group& g, const double* dP);
template <typename T>
int push_vector(snk_ctx* c, std::vector<T>& v, const T** dptr);

// test hook: 0 runs the F-row test on every function (no block prefilter)
int g_frow_prefilter = 1;

// Steps of one batch group up to G: Eq. collocation, Eq. fmat, the screen (when enabled),
// Eqs. 3c_grid + gmat.
// Eq. collocation and Eq. fmat for one batch group: Phi_g, then F_g = P[:, B_g] Phi_g.
int group_F(snk_ctx* c, const Group& g, const double* dP, bool timed)
{
    hipStream_t s = c->stream;
    const int64_t nbf = c->nbf;
    if (timed) HIPCHECK(c, hipEventRecord(c->ev[0], s));
    // Eq. collocation for every tile in one launch: Phi_t (nB x ncols_t, row stride ncols_t)
    {
        std::vector<CollTile> ct;
        for (const Tile& t : g.tiles) {
            if (t.coll_shells.empty()) continue;
            CollTile r{};
            r.col0 = t.col0;
            r.ncols = t.ncols;
            r.phi_off = t.phi_off;
            r.shells = t.d_coll_shells;
            r.rows = t.d_coll_rows;
            r.nsh = (int32_t)t.coll_shells.size();
            ct.push_back(r);
        }
        const int64_t nwg = collocate_tiles_plan(ct.data(), (int32_t)ct.size());
        if (!ct.empty()) {
            const CollTile* d = nullptr;
            int rc = push_vector(c, ct, &d);
            if (rc) return rc;
            const int64_t off = (int64_t)g.b0 * kBatch;
            if (c->mixed)
                HIPCHECK(c, launch_collocate_tiles(c->d_px + off, c->d_py + off, c->d_pz + off, c->d_shells, c->d_exps,
                                                   c->d_coefs, d, (int32_t)ct.size(), nwg, c->d_Phi32, s));
            else
                HIPCHECK(c, launch_collocate_tiles(c->d_px + off, c->d_py + off, c->d_pz + off, c->d_shells, c->d_exps,
                                                   c->d_coefs, d, (int32_t)ct.size(), nwg, c->d_Phi, s));
        }
    }
    if (timed) HIPCHECK(c, hipEventRecord(c->ev[1], s));
    const int ntile = (int)g.tiles.size();
    if (c->frow_restrict) {
        // rows L_t of F that can reach eps_basis on the tile: functions whose bound
        // sum_{nu in B_t} |P_lam,nu| max_i |Phi_nu,i| >= eps_basis, by whole shells
        HIPCHECK(c, launch_fill(c->d_fflag, (int64_t)ntile * c->nshell, 0, s));
        const Tile& last = g.tiles.back();
        const int64_t nfull = last.row_off;
        const int64_t ncols_full = ntile > 1 ? g.tiles[0].ncols : 0;
        if (c->mixed)
            HIPCHECK(c, launch_row_absmax(c->d_Phi32, nfull, ncols_full, g.phi_rows, last.ncols, c->d_mx, s));
        else
            HIPCHECK(c, launch_row_absmax(c->d_Phi, nfull, ncols_full, g.phi_rows, last.ncols, c->d_mx, s));
        if (c->d_pmax && g_frow_prefilter) {
            // the block maxima of |P| once per build (every caller runs the groups from the
            // first), then per tile the functions the block bound cannot rule out
            if (&g == &c->groups.front())
                HIPCHECK(c, launch_pblock_max(dP, nbf, c->d_blk_fn0, c->nblk, c->d_pmax, s));
            HIPCHECK(c, launch_ftilde_cand(g.d_fn_cat, g.d_roff, c->d_mx, ntile, c->d_fn_blk, c->d_blk_fn0, c->nblk,
                                           c->d_pmax, c->opts.eps_basis, nbf, c->d_cand, nbf, c->d_ncand, s));
            HIPCHECK(c, launch_ftilde_flag(dP, nbf, g.d_fn_cat, g.d_roff, ntile, c->d_mx, c->opts.eps_basis,
                                           c->d_fn_shell, c->nshell, c->d_fflag, s, c->d_cand, nbf, c->d_ncand));
        } else {
            HIPCHECK(c, launch_ftilde_flag(dP, nbf, g.d_fn_cat, g.d_roff, ntile, c->d_mx, c->opts.eps_basis,
                                           c->d_fn_shell, c->nshell, c->d_fflag, s));
        }
        if (c->split) {
            HIPCHECK(c, launch_partition(c->d_mx, g.d_fn_cat, g.d_roff, ntile, kWeakPhi, c->d_perm, c->d_cperm,
                                         c->d_nstrong, s));
            c->tile_nstrong.assign(ntile, 0);
            HIPCHECK(c, hipMemcpyAsync(c->tile_nstrong.data(), c->d_nstrong, ntile * sizeof(int32_t),
                                       hipMemcpyDeviceToHost, s));
        }
        HIPCHECK(c, launch_tile_rows(c->d_fflag, ntile, c->nshell, c->d_shell_l, c->d_shell_row, c->nbf, c->d_frows,
                                     c->d_fcount, s));
        c->tile_frows.assign(ntile, 0);
        HIPCHECK(c, hipMemcpyAsync(c->tile_frows.data(), c->d_fcount, ntile * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHECK(c, hipStreamSynchronize(s));
    }
    // Eq. fmat for every tile in one grouped launch: F[L_t, tile columns] = P[L_t, B_t] Phi_t
    int rc = group_fgemm(c, g, dP);
    if (rc) return rc;
    if (timed) HIPCHECK(c, hipEventRecord(c->ev[2], s));
    return SNK_OK;
}

// Copies n records into the device arena and returns their device address.  The host mirror
// of a record is never rewritten before the stream has passed the copy that reads it: when the
// arena is full the stream is drained and the arena restarts (larger if needed).
int push_records(snk_ctx* c, const void* src, size_t bytes, const void** dptr)
{
    bytes = (bytes + 255) & ~(size_t)255;
    if (c->arena_cur + bytes > c->h_arena.size()) {
        // every stream of the context may still read records: wait for the device
        HIPCHECK(c, hipDeviceSynchronize());
        if (bytes > c->h_arena.size()) {
            const size_t cap = std::max<size_t>(bytes, std::max<size_t>((size_t)1 << 20, 2 * c->h_arena.size()));
            (void)hipFree(c->d_arena);
            c->d_arena = nullptr;
            HIPCHECK(c, hipMalloc((void**)&c->d_arena, cap));
            c->h_arena.assign(cap, 0);
        }
        c->arena_cur = 0;
    }
    char* h = c->h_arena.data() + c->arena_cur;
    std::memcpy(h, src, bytes);   // bytes is rounded up: the source is padded by the callers' vectors
    HIPCHECK(c, hipMemcpyAsync(c->d_arena + c->arena_cur, h, bytes, hipMemcpyHostToDevice, c->stream));
    *dptr = c->d_arena + c->arena_cur;
    c->arena_cur += bytes;
    return SNK_OK;
}

template <typename T>
int push_vector(snk_ctx* c, std::vector<T>& v, const T** dptr)
{
    const size_t n = v.size();
    v.resize(n + (256 + sizeof(T) - 1) / sizeof(T));   // padding read by the rounded copy
    const void* d = nullptr;
    const int rc = push_records(c, v.data(), n * sizeof(T), &d);
    v.resize(n);
    *dptr = static_cast<const T*>(d);
    return rc;
}

enum GemmKind { kGemmF64 = 0, kGemmF32 = 1, kGemmF32dA = 2, kGemmF32dd = 3, kGemmSplit = 4 };

int launch_gemm_list(snk_ctx* c, std::vector<GemmProb>& probs, GemmKind kind, bool bt)
{
    if (probs.empty()) return SNK_OK;
    int64_t nwg = 0;
    const int asz = kind == kGemmF32 ? 4 : 8, bsz = (kind == kGemmF64 || kind == kGemmF32dd || kind == kGemmSplit) ? 8 : 4;
    int tile;
    if (kind == kGemmSplit) {
        // split products: the tile for the whole sum over both precisions
        std::vector<GemmProb> full(probs);
        for (auto& p : full) p.K += p.K2;
        tile = ggemm_tile(full.data(), (int)full.size());
    } else {
        tile = ggemm_tile(probs.data(), (int)probs.size());
    }
    for (auto& p : probs) {
        ggemm_plan(p, tile, asz, bsz);
        p.wg0 = nwg;
        nwg += ggemm_workgroups(p);
    }
    const GemmProb* d = nullptr;
    int rc = push_vector(c, probs, &d);
    if (rc) return rc;
    const int n = (int)probs.size();
    hipError_t e = kind == kGemmF64    ? launch_ggemm_f64(d, n, nwg, tile, bt, c->stream)
                   : kind == kGemmF32  ? launch_ggemm_f32(d, n, nwg, tile, bt, c->stream)
                   : kind == kGemmF32dA ? launch_ggemm_f32_dA(d, n, nwg, tile, bt, c->stream)
                   : kind == kGemmF32dd ? launch_ggemm_f32_dd(d, n, nwg, tile, bt, c->stream)
                                        : launch_gsplit(d, n, nwg, tile, c->stream);
    HIPCHECK(c, e);
    return SNK_OK;
}

// The products in probs (all read B the same way) in grouped launches on the context's stream.
// FP32 kinds keep every FP32 sum within kFp32MaxK terms: split products must already have
// chunks that short; a product written in one piece longer than that is cut into k slices, one
// launch per slice, the later slices added into C.
int run_gemms(snk_ctx* c, std::vector<GemmProb>& probs, GemmKind kind, bool bt)
{
    if (kind == kGemmF64 || kind == kGemmSplit) return launch_gemm_list(c, probs, kind, bt);
    const int asz = kind == kGemmF32 ? 4 : 8, bsz = (kind == kGemmF64 || kind == kGemmF32dd) ? 8 : 4;
    std::vector<std::vector<GemmProb>> slices(1);
    for (const GemmProb& p : probs) {
        if (p.ksplit > 1) {
            if ((p.K + p.ksplit - 1) / p.ksplit > kFp32MaxK) {
                set_err(c, "internal: FP32 product chunk longer than the FP32 sum limit");
                return SNK_E_DEVICE;
            }
            slices[0].push_back(p);
            continue;
        }
        for (int64_t k0 = 0, sl = 0; k0 < std::max<int64_t>(1, p.K); k0 += kFp32MaxK, ++sl) {
            GemmProb q = p;
            q.K = (int32_t)std::min<int64_t>(kFp32MaxK, p.K - k0);
            if (k0 > 0) {
                if (q.acol) q.acol += k0;
                else q.A = (const char*)p.A + k0 * asz;
                if (bt) q.B = (const char*)p.B + k0 * bsz;
                else if (q.bmap) q.bmap += k0;
                else q.B = (const char*)p.B + k0 * p.ldb * bsz;
                q.vec |= kGemmAccumulate;
            }
            if ((size_t)sl >= slices.size()) slices.resize(sl + 1);
            slices[sl].push_back(q);
        }
    }
    for (auto& sl : slices) {
        int rc = launch_gemm_list(c, sl, kind, bt);
        if (rc) return rc;
    }
    return SNK_OK;
}

// T[r][ccol(n)] += sum_z part[tile][z][rinv(r)][n] for the tiles in list order (rows of T: nbf)
int run_reduce(snk_ctx* c, std::vector<RedTile>& tiles, double* T)
{
    if (tiles.empty()) return SNK_OK;
    const RedTile* d = nullptr;
    int rc = push_vector(c, tiles, &d);
    if (rc) return rc;
    HIPCHECK(c, launch_group_reduce(c->d_part, d, (int)tiles.size(), T, c->nbf, c->nbf, c->stream));
    return SNK_OK;
}

// The split partial-product buffer holds at least n elements (the stream is drained before
// a smaller buffer is replaced).
int ensure_part(snk_ctx* c, int64_t n)
{
    if (n <= c->part_elems) return SNK_OK;
    if (c->pipe) {
        set_err(c, "partial-product buffer too small for an overlapped build");
        return SNK_E_DEVICE;
    }
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    (void)hipFree(c->d_part);
    c->d_part = nullptr;
    const int64_t cap = std::max<int64_t>(n, c->part_elems + c->part_elems / 2);
    int rc = dalloc(c, &c->d_part, (size_t)cap);
    if (rc) {
        c->part_elems = 0;
        return rc;
    }
    c->part_elems = cap;
    return SNK_OK;
}

// Chunks over k for a set of products with otiles output tiles in all: enough workgroups for
// the device, chunks of whole batches, at most 256.
int choose_ksplit(int64_t otiles, int64_t batches)
{
    const int64_t ks = (kGemmTarget + std::max<int64_t>(1, otiles) - 1) / std::max<int64_t>(1, otiles);
    return (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(ks, 256), std::max<int64_t>(1, batches)));
}

int64_t out_tiles(int64_t M, int64_t N) { return ((M + 127) / 128) * ((N + 127) / 128); }

// Grows a device buffer to at least n bytes (the stream is drained before a smaller buffer is
// replaced).
int ensure_bytes(snk_ctx* c, void** p, size_t* cap, size_t n)
{
    if (n <= *cap && *p) return SNK_OK;
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    (void)hipFree(*p);
    *p = nullptr;
    const size_t sz = std::max<size_t>(n, *cap + *cap / 2);
    hipError_t e = hipMalloc(p, std::max<size_t>(sz, 256));
    if (e != hipSuccess) {
        *p = nullptr;
        *cap = 0;
        set_err(c, std::string("hipMalloc: ") + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? SNK_E_NOMEM : SNK_E_DEVICE;
    }
    *cap = std::max<size_t>(sz, 256);
    return SNK_OK;
}

// run_gemms between the timing events of product kind `slot` (timed builds)
int timed_gemms(snk_ctx* c, int slot, std::vector<GemmProb>& probs, GemmKind kind, bool bt)
{
    if (probs.empty()) return SNK_OK;
    if (c->timing) HIPCHECK(c, hipEventRecord(c->gev[2 * slot], c->stream));
    int rc = run_gemms(c, probs, kind, bt);
    if (rc) return rc;
    if (c->timing) {
        HIPCHECK(c, hipEventRecord(c->gev[2 * slot + 1], c->stream));
        c->gl[slot] = true;
    }
    return SNK_OK;
}

// Eq. fmat for group g: F[L_t, tile columns] = P[L_t, B_t] Phi_t for every tile, with the rows
// written straight into F.  Where a tile does not take every row and column of P, P[L_t, B_t]
// is gathered first for all tiles in one launch.  One grouped launch computes every tile's
// product.  Split build: the strong functions' columns of P are gathered in FP64, the weak
// ones in FP32 together with the weak rows of Phi_t, and each tile's product is FP64 over the
// strong functions plus FP32 matrix cores over the weak ones, written once.
int group_fgemm(snk_ctx* c, const Group& g, const double* dP)
{
    const int64_t nbf = c->nbf;
    const int64_t ld = g.ncols;
    const size_t esz = c->mixed ? sizeof(float) : sizeof(double);
    // rows outside L_t are zero; they are written only where a reader takes every row (no
    // density screen, training data, debugging): the screens give those shells U = 0 without
    // reading them and never list their blocks
    const bool zero_rows = c->opts.screen == SNK_SCREEN_NONE || c->zero_f_rows;
    bool need_zero = false;
    std::vector<GatherTile> gt, gw, gphi;
    std::vector<int64_t> pc_off(g.tiles.size(), -1), pw_off(g.tiles.size(), -1), phw_off(g.tiles.size(), -1);
    int64_t pc_elems = 0, pw_elems = 0, phw_elems = 0;
    int32_t max_rows = 0, max_wrows = 0;
    for (size_t ti = 0; ti < g.tiles.size(); ++ti) {
        const Tile& t = g.tiles[ti];
        const int64_t L = c->frow_restrict ? c->tile_frows[ti] : nbf;
        c->acc_fn += (double)t.nB * t.ncols;
        c->acc_frows += (double)L * t.ncols;
        c->acc_cols += (double)t.ncols;
        if (t.nB == 0 || L == 0 || L < nbf) need_zero |= zero_rows;
        if (t.nB == 0 || L == 0) continue;
        if (L < nbf || !t.all_functions || c->split) {
            const int32_t ns = c->split ? c->tile_nstrong[ti] : t.nB;
            GatherTile q{};
            q.src_ld = nbf;
            q.rows = L < nbf ? c->d_frows + (int64_t)ti * nbf : nullptr;
            q.cols = c->split ? c->d_cperm + t.row_off : (t.all_functions ? nullptr : t.d_coll_fn);
            q.M = (int32_t)L;
            q.N = ns;
            q.ld = (ns + 3) & ~3;   // 16-byte aligned rows for the vector loads of the product
            q.out_off = pc_elems;
            pc_off[ti] = pc_elems;
            pc_elems += L * q.ld;
            max_rows = std::max<int32_t>(max_rows, (int32_t)L);
            if (ns > 0) gt.push_back(q);
            if (ns < t.nB) {
                // the weak columns of P and the weak rows of Phi_t, rounded to FP32
                GatherTile w = q;
                w.cols = q.cols + ns;
                w.N = t.nB - ns;
                w.ld = (w.N + 3) & ~3;
                w.out_off = pw_elems;
                pw_off[ti] = pw_elems;
                pw_elems += L * w.ld;
                gw.push_back(w);
                GatherTile f{};
                f.src_off = t.phi_off;
                f.src_ld = t.ncols;
                f.rows = c->d_perm + t.row_off + ns;
                f.M = t.nB - ns;
                f.N = (int32_t)t.ncols;
                f.ld = (int32_t)t.ncols;
                f.out_off = phw_elems;
                phw_off[ti] = phw_elems;
                phw_elems += (int64_t)f.M * t.ncols;
                max_wrows = std::max<int32_t>(max_wrows, f.M);
                gphi.push_back(f);
            }
        }
    }
    if (need_zero) {
        if (c->mixed) HIPCHECK(c, launch_fill(c->d_F32, nbf * ld, 0.0f, c->stream));
        else HIPCHECK(c, launch_fill(c->d_F, nbf * ld, 0.0, c->stream));
    }
    c->tile_phw_off = phw_off;
    int rc = SNK_OK;
    if (!gt.empty()) {
        if ((rc = ensure_bytes(c, &c->d_Pc, &c->pc_bytes, (size_t)pc_elems * esz))) return rc;
        const GatherTile* d = nullptr;
        if ((rc = push_vector(c, gt, &d))) return rc;
        if (c->mixed)
            HIPCHECK(c, launch_gather_tiles(c->d_P32, d, (int)gt.size(), max_rows, (float*)c->d_Pc, c->stream));
        else
            HIPCHECK(c, launch_gather_tiles(dP, d, (int)gt.size(), max_rows, (double*)c->d_Pc, c->stream));
    }
    if (!gw.empty()) {
        if ((rc = ensure_bytes(c, &c->d_Pw, &c->pw_bytes, (size_t)pw_elems * sizeof(float)))) return rc;
        if ((rc = ensure_bytes(c, &c->d_Phw, &c->phw_bytes, (size_t)phw_elems * sizeof(float)))) return rc;
        const GatherTile* d = nullptr;
        if ((rc = push_vector(c, gw, &d))) return rc;
        HIPCHECK(c, launch_gather_tiles(dP, d, (int)gw.size(), max_rows, (float*)c->d_Pw, c->stream));
        if ((rc = push_vector(c, gphi, &d))) return rc;
        HIPCHECK(c, launch_gather_tiles(c->d_Phi, d, (int)gphi.size(), max_wrows, (float*)c->d_Phw, c->stream));
    }
    std::vector<GemmProb> probs, split;
    for (size_t ti = 0; ti < g.tiles.size(); ++ti) {
        const Tile& t = g.tiles[ti];
        const int64_t L = c->frow_restrict ? c->tile_frows[ti] : nbf;
        if (t.nB == 0 || L == 0) continue;
        const int32_t ns = c->split ? c->tile_nstrong[ti] : t.nB;
        GemmProb p{};
        if (pc_off[ti] >= 0) {
            p.A = (const char*)c->d_Pc + pc_off[ti] * esz;
            p.lda = (ns + 3) & ~3;
        } else {
            p.A = c->mixed ? (const void*)c->d_P32 : (const void*)dP;
            p.lda = nbf;
        }
        p.B = c->mixed ? (const void*)(c->d_Phi32 + t.phi_off) : (const void*)(c->d_Phi + t.phi_off);
        p.bmap = c->split ? c->d_perm + t.row_off : nullptr;
        p.ldb = t.ncols;
        p.C = c->mixed ? (void*)(c->d_F32 + t.col0) : (void*)(c->d_F + t.col0);
        p.crow = L < nbf ? c->d_frows + (int64_t)ti * nbf : nullptr;
        p.ldc = ld;
        p.M = (int32_t)L;
        p.N = (int32_t)t.ncols;
        p.K = ns;
        p.ksplit = 1;
        const double f_strong = 2.0 * (double)L * (double)t.ncols * (double)ns;
        if (ns < t.nB) {
            p.A2 = (const char*)c->d_Pw + pw_off[ti] * sizeof(float);
            p.lda2 = (t.nB - ns + 3) & ~3;
            p.B2 = (const char*)c->d_Phw + phw_off[ti] * sizeof(float);
            p.ldb2 = t.ncols;
            p.K2 = t.nB - ns;
            const double f_weak = 2.0 * (double)L * (double)t.ncols * (double)(t.nB - ns);
            c->acc_flops64 += f_strong;
            c->acc_flops32 += f_weak;
            c->slot_flops[1][0] += f_strong;
            c->slot_flops[1][1] += f_weak;
            split.push_back(p);
        } else {
            (c->mixed ? c->acc_flops32 : c->acc_flops64) += f_strong;
            c->slot_flops[c->mixed ? 1 : 0][c->mixed ? 1 : 0] += f_strong;
            probs.push_back(p);
        }
    }
    if ((rc = timed_gemms(c, c->mixed ? 1 : 0, probs, c->mixed ? kGemmF32 : kGemmF64, false))) return rc;
    return timed_gemms(c, 1, split, kGemmSplit, false);
}

// Eq. usym_k for group g: Kt[M_t, B_t] += G[M_t, tile columns] Phi_t^T for every tile in one
// grouped launch (split over points where the tiles are few), then one fixed-order reduction
// of all tiles into Kt.  M_t: the rows of the tile's kept blocks (screen with basis screening;
// every other row of G is zero on the tile), else every row.
int group_K(snk_ctx* c, const Group& g)
{
    const int64_t nbf = c->nbf;
    const int64_t ld = g.ncols;
    const bool restrict_rows = c->row_restrict && c->tile_rows.size() == g.tiles.size();
    const int ntile = (int)g.tiles.size();
    int64_t otiles = 0;
    int32_t max_rows = 0;
    for (int ti = 0; ti < ntile; ++ti) {
        const Tile& t = g.tiles[ti];
        const int64_t M = restrict_rows ? c->tile_rows[ti] : nbf;
        if (restrict_rows) c->acc_grows += (double)M * t.ncols;
        max_rows = std::max<int32_t>(max_rows, (int32_t)M);
        if (t.nB > 0 && M > 0) otiles += out_tiles(M, t.nB);
    }
    if (otiles == 0) return SNK_OK;
    int64_t need = 0;
    std::vector<int> ks(ntile, 1);
    for (int ti = 0; ti < ntile; ++ti) {
        const Tile& t = g.tiles[ti];
        const int64_t M = restrict_rows ? c->tile_rows[ti] : nbf;
        if (t.nB == 0 || M == 0) continue;
        ks[ti] = c->pipe ? c->nsplit : choose_ksplit(otiles, t.b1 - t.b0);
        // FP32 products (legacy FP32 storage, or the weak columns of the split build): chunks
        // of at most kFp32MaxK points, added in FP64 by the reduction
        if (c->mixed || c->split)
            ks[ti] = std::max<int>(ks[ti], (int)((t.ncols + kFp32MaxK - 1) / kFp32MaxK));
        need += (int64_t)ks[ti] * M * t.nB;
    }
    int rc = ensure_part(c, need);
    if (rc) return rc;
    if (restrict_rows)
        HIPCHECK(c, launch_rinv(c->d_trows, nbf, nullptr, c->d_tcount, ntile, nbf, max_rows, c->d_rinv, c->stream));
    std::vector<GemmProb> probs, weak;
    std::vector<RedTile> red;
    int64_t poff = 0;
    for (int ti = 0; ti < ntile; ++ti) {
        const Tile& t = g.tiles[ti];
        const int64_t M = restrict_rows ? c->tile_rows[ti] : nbf;
        if (t.nB == 0 || M == 0) continue;
        // split build: product columns in the tile's strong-then-weak order; the FP64 product
        // takes the strong columns rounded up to whole 64-column blocks (its output tiles would
        // pad them anyway), so the first weak columns leave the FP32 product
        const int32_t ns0 = c->split ? c->tile_nstrong[ti] : t.nB;
        const int32_t ns = c->split ? std::min<int32_t>(t.nB, (ns0 + 63) / 64 * 64) : t.nB;
        GemmProb p{};
        p.A = c->d_G + t.col0;
        p.lda = ld;
        p.arow = restrict_rows ? c->d_trows + (int64_t)ti * nbf : nullptr;
        p.B = c->mixed ? (const void*)(c->d_Phi32 + t.phi_off) : (const void*)(c->d_Phi + t.phi_off);
        p.bmap = c->split ? c->d_perm + t.row_off : nullptr;
        p.ldb = t.ncols;
        p.C = c->d_part + poff;
        p.ldc = t.nB;
        p.cstride = M * t.nB;
        p.M = (int32_t)M;
        p.N = ns;
        p.K = (int32_t)t.ncols;
        p.ksplit = ks[ti];
        if (ns > 0) probs.push_back(p);
        (c->mixed ? c->acc_flops32 : c->acc_flops64) += 2.0 * (double)M * (double)ns * (double)t.ncols;
        c->slot_flops[c->mixed ? 3 : 2][c->mixed ? 1 : 0] += 2.0 * (double)M * (double)ns * (double)t.ncols;
        if (ns < t.nB) {
            // the weak rows of Phi_t as the F product left them in FP32 (rows in weak order)
            GemmProb q = p;
            q.B = (const char*)c->d_Phw + (c->tile_phw_off[ti] + (int64_t)(ns - ns0) * t.ncols) * sizeof(float);
            q.bmap = nullptr;
            q.C = c->d_part + poff + ns;
            q.N = t.nB - ns;
            weak.push_back(q);
            c->acc_flops32 += 2.0 * (double)M * (double)(t.nB - ns) * (double)t.ncols;
            c->slot_flops[3][1] += 2.0 * (double)M * (double)(t.nB - ns) * (double)t.ncols;
        }
        RedTile r{};
        r.poff = poff;
        r.M = (int32_t)M;
        r.N = t.nB;
        r.ksplit = ks[ti];
        r.rinv = restrict_rows ? c->d_rinv + (int64_t)ti * nbf : nullptr;
        r.ccol = c->split ? c->d_cperm + t.row_off : (t.all_functions ? nullptr : t.d_coll_fn);
        red.push_back(r);
        poff += (int64_t)ks[ti] * M * t.nB;
    }
    if ((rc = timed_gemms(c, c->mixed ? 3 : 2, probs, c->mixed ? kGemmF32dA : kGemmF64, true))) return rc;
    if ((rc = timed_gemms(c, 3, weak, kGemmF32dA, true))) return rc;
    if ((rc = run_reduce(c, red, c->d_Kt))) return rc;
    if (c->split && restrict_rows) {
        // rigorous bound on the energy moved by the FP32 products of the group (accumulated
        // over the build): sum over tiles and G rows of |G row| (sum of |P| over weak columns)
        std::vector<BoundTile> bt;
        for (int ti = 0; ti < ntile; ++ti) {
            const Tile& t = g.tiles[ti];
            bt.push_back(BoundTile{t.col0, (int32_t)t.ncols, t.row_off, t.nB, c->tile_nstrong[ti]});
        }
        const BoundTile* d = nullptr;
        if ((rc = push_vector(c, bt, &d))) return rc;
        HIPCHECK(c, launch_lowprec_bound(c->d_G, ld, c->d_P_cur, nbf, d, ntile, c->d_trows, c->d_tcount, c->d_cperm,
                                         c->d_lpb, c->d_lpb + (int64_t)c->max_group_tiles * kBoundChunksPerTile,
                                         c->stream));
    }
    return SNK_OK;
}

// U (bound factors) and N (F norms) of every shell on every batch of the group
int group_bounds(snk_ctx* c, const Group& g)
{
    const int64_t off = (int64_t)g.b0 * kBatch;
    const int nb = g.b1 - g.b0;
    const int ntile = (int)g.tiles.size();
    hipStream_t s = c->stream;
    c->bound_order.clear();
    DiagArgs a{};
    a.px = c->d_px + off;
    a.py = c->d_py + off;
    a.pz = c->d_pz + off;
    a.pw = c->d_pw + off;
    a.F = c->d_F;
    a.F32 = c->mixed ? c->d_F32 : nullptr;
    a.ld = g.ncols;
    a.prims = c->d_dprims32;
    a.U = c->d_U;
    a.lun = c->d_lun;
    a.fmax = nullptr;   // the sn-LinK F-tilde is formed from |P| and Phi-tilde instead
    a.nshell = c->nshell;
    a.nbatch = nb;
    a.tab = c->d_boys;
    a.tile_batches = c->tile_batches;
    if (c->frow_restrict) {
        // only the shells whose F rows a tile computed have F != 0 there: list them per tile,
        // evaluate those, and give every other shell U = 0 (log features -40, as for U = 0)
        if (!c->d_dcount) {
            int rc;
            for (int l = 0; l < 3; ++l)
                if ((rc = dalloc(c, &c->d_dlist[l], (size_t)c->max_group_tiles * std::max(1, c->n_diag[l]))))
                    return rc;
            if ((rc = dalloc(c, &c->d_dcount, (size_t)3 * c->max_group_tiles))) return rc;
        }
        DiagLists d{};
        for (int l = 0; l < 3; ++l) {
            d.dsh[l] = c->d_diag_sh[l];
            d.n[l] = c->n_diag[l];
            d.list[l] = c->d_dlist[l];
            d.count[l] = c->d_dcount + (int64_t)l * c->max_group_tiles;
        }
        HIPCHECK(c, launch_diag_lists(d, c->d_fflag, ntile, c->nshell, s));
        HIPCHECK(c, launch_fill(c->d_U, (int64_t)nb * c->nshell, 0.0, s));
        if (c->d_lun) HIPCHECK(c, launch_fill(reinterpret_cast<float*>(c->d_lun), (int64_t)2 * nb * c->nshell, -40.0f, s));
        if ((int)c->tile_frows.size() == ntile && ntile > 1 && c->tile_batches > 0) {
            // the batches of the tiles with the most F rows (a tile's listed shells) first, in
            // decreasing powers of two: each batch writes only its own U, so the order only
            // schedules the heavy workgroups ahead of the launches' tails
            std::vector<int32_t> order(nb);
            std::vector<uint8_t> key(nb);
            int32_t cnt[32] = {}, pos[32];
            for (int j = 0; j < nb; ++j) {
                const int t = std::min(ntile - 1, j / c->tile_batches);
                key[j] = (uint8_t)__builtin_clz((uint32_t)std::max(0, c->tile_frows[t]) + 1u);
                ++cnt[key[j]];
            }
            for (int q = 0, p = 0; q < 32; ++q) {
                pos[q] = p;
                p += cnt[q];
            }
            for (int j = 0; j < nb; ++j) order[pos[key[j]]++] = j;
            int rc = push_vector(c, order, &a.batch_order);
            if (rc) return rc;
            c->bound_order = std::move(order);   // also the order of the estimate and count passes
        }
    }
    for (int l = 0; l < 3; ++l) {
        a.dsh = c->d_diag_sh[l];
        a.drow = c->d_diag_row[l];
        a.dpb = c->d_diag_pb[l];
        a.dnp = c->d_diag_np[l];
        a.n = c->n_diag[l];
        a.list = c->frow_restrict ? c->d_dlist[l] : nullptr;
        a.count = c->frow_restrict ? c->d_dcount + (int64_t)l * c->max_group_tiles : nullptr;
        HIPCHECK(c, launch_diag_bound(l, a, s));
    }
    return SNK_OK;
}

// Eq. exx_fmat_approx for every batch of group g: Phi-tilde per batch and tile row, then one
// grouped product over the tiles, Ft[b][mu] = sum_{nu in B_t} Phi~[b][nu] |P|[nu][mu] with mu over
// the whole basis, then F-tilde per shell (the largest over its functions) into d_fmax.
// |P| (d_Pabs) is formed once per build.
int link_ftilde(snk_ctx* c, const Group& g)
{
    hipStream_t s = c->stream;
    const int64_t nbf = c->nbf;
    const int nb = g.b1 - g.b0;
    const int ntile = (int)g.tiles.size();
    const int64_t off = (int64_t)g.b0 * kBatch;
    HIPCHECK(c, launch_phimax(c->mixed ? nullptr : c->d_Phi, c->mixed ? c->d_Phi32 : nullptr, g.d_roff, ntile,
                              c->tile_batches, g.tiles.back().ncols, c->d_pw + off, nb, c->d_phimax, c->link_ld, s));
    std::vector<GemmProb> probs;
    bool empty = false;
    for (const Tile& t : g.tiles) {
        if (t.nB == 0) {
            empty = true;
            continue;
        }
        GemmProb p{};
        p.A = c->d_phimax + (int64_t)(t.b0 - g.b0) * c->link_ld;
        p.lda = c->link_ld;
        p.B = c->d_Pabs;
        p.bmap = t.all_functions ? nullptr : t.d_coll_fn;
        p.ldb = nbf;
        p.C = c->d_FtT + (int64_t)(t.b0 - g.b0) * nbf;
        p.ldc = nbf;
        p.M = t.b1 - t.b0;
        p.N = (int32_t)nbf;
        p.K = t.nB;
        p.ksplit = 1;
        probs.push_back(p);
    }
    if (empty) HIPCHECK(c, launch_fill(c->d_FtT, (int64_t)nb * nbf, 0.0, s));   // tiles without functions
    int rc = launch_gemm_list(c, probs, kGemmF64, false);
    if (rc) return rc;
    HIPCHECK(c, launch_shellmax(c->d_FtT, nbf, c->d_shell_l, c->d_shell_row, c->nshell, nb, c->d_fmax, s));
    return SNK_OK;
}

// |P| for the sn-LinK estimates of this build
int link_prepare(snk_ctx* c, const double* dP)
{
    if (c->opts.screen != SNK_SCREEN_LINK || !c->d_Pabs) return SNK_OK;
    HIPCHECK(c, launch_abs(dP, c->nbf * c->nbf, c->d_Pabs, c->stream));
    return SNK_OK;
}

// Testing: decodes the run and B-task records the screen wrote for group g into
// (batch, A, B) triples of kept shell pairs (c->kept).
int capture_kept(snk_ctx* c, const Group& g, const int64_t* total_runs, const std::vector<int64_t>& bt_base)
{
    const int nb = g.b1 - g.b0;
    std::vector<int32_t> shell_of(c->nbf, -1);
    for (int sh = 0; sh < c->nshell; ++sh) shell_of[c->sfn[sh]] = sh;
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    c->kept.clear();
    for (int k = 0; k < c->nlist; ++k) {
        const int TA = kListTile(k), RS = 2 + TA, BS = 2 + 2 * TA;
        const int64_t nrun = total_runs[k], nbt = bt_base[(size_t)k * (nb + 1) + nb];
        if (nrun == 0) continue;
        std::vector<int32_t> runs((size_t)nrun * RS), bts((size_t)nbt * BS), bro(nb + 1);
        HIPCHECK(c, hipMemcpy(runs.data(), c->d_pool_runs[k], runs.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIPCHECK(c, hipMemcpy(bts.data(), c->d_pool_bt[k], bts.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIPCHECK(c, hipMemcpy(bro.data(), c->d_bro[k], bro.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int j = 0; j < nb; ++j)
            for (int32_t r = bro[j]; r < bro[j + 1]; ++r) {
                const int32_t* rec = &runs[(size_t)r * RS];
                for (int32_t q = rec[0]; q < rec[1]; ++q) {
                    const int32_t* bt = &bts[(size_t)q * BS];
                    for (int a = 0; a < TA; ++a)
                        if (bt[1] & (1 << a)) {
                            c->kept.push_back(g.b0 + j);
                            c->kept.push_back(shell_of[rec[2 + a]]);
                            c->kept.push_back(shell_of[bt[0]]);
                        }
                }
            }
    }
    return SNK_OK;
}

int group_until_G(snk_ctx* c, const Group& g, const double* dP, bool timed, GroupStats* gs, float* yraw = nullptr)
{
    hipStream_t s = c->stream;
    const int64_t nbf = c->nbf;
    const int64_t ld = g.ncols;
    const int64_t off = (int64_t)g.b0 * kBatch;
    const int nb = g.b1 - g.b0;
    const bool screen = c->opts.screen != SNK_SCREEN_NONE;
    {
        int rc = group_F(c, g, dP, timed);
        if (rc) return rc;
    }

    int64_t gpts = 0;
    std::vector<int64_t> npts(nb);
    for (int b = g.b0; b < g.b1; ++b) {
        npts[b - g.b0] = c->batch_npts[b];
        gpts += c->batch_npts[b];
    }
    for (int cl = 0; cl < 6; ++cl) gs->cand += c->ntask[cl] * gpts;
    int64_t total_runs[12] = {};
    // screened lists: per list the batches with runs, in decreasing powers of two of their B
    // tasks (batches write disjoint columns of G, so the order only schedules the heavy
    // workgroups ahead of the launch's tail; a bucket pass keeps the host's share, which the
    // device waits for, linear), one upload for all lists
    std::vector<int32_t> order;
    int64_t order_off[12] = {};
    int32_t order_cnt[12] = {};
    const int32_t* d_order = nullptr;
    if (screen) {
        if (timed) HIPCHECK(c, hipEventRecord(c->ev[7], s));
        {
            int rc = group_bounds(c, g);
            if (rc) return rc;
        }
        const bool link = c->opts.screen == SNK_SCREEN_LINK;
        // the link selection has per-pair thresholds instead of an energy budget
        const double eps_batch = link ? 0.0 : c->opts.eps_skip_energy / std::max(1, c->nbatch);
        // FP32 blocks: estimates summing to at most eps_lowprec / kLowRelErr per build
        const double eps_low =
            c->nlist == 12 ? c->opts.eps_lowprec_energy / kLowRelErr / std::max(1, c->nbatch) : 0.0;
        if (c->mlp) {
            EstArgs ea{};
            ea.U = c->d_U;
            ea.lun = c->d_lun;
            ea.nshell = c->nshell;
            ea.nbatch = nb;
            ea.shell_l = c->d_shell_l;
            ea.nne = (int64_t)c->ne_list.size();
            ea.ne_p = c->d_ne_list;
            ea.ne_ab = c->d_ne_ab;
            ea.ne_feat = c->d_ne_feat;
            ea.ne_lp = c->d_lp;
            ea.ne_pos = c->d_ne_pos;
            ea.geo = c->d_geo + g.b0;
            ea.eps_batch = eps_batch;
            ea.params = mlp_params(c->mlp);
            ea.norm = mlp_norm(c->mlp);
            int hr = 0;
            mlp_range(c->mlp, ea.lo, ea.hi, &ea.margin, &hr);
            ea.est = c->d_est;
            ea.yraw = yraw;
            ea.thr = c->d_thr;
            ea.eps_low = eps_low;
            ea.thr2 = c->d_thr2;
            ea.skipped = c->d_skipped;
            if ((int)c->bound_order.size() == nb) {
                int rc = push_vector(c, c->bound_order, &ea.batch_order);   // read by this launch only
                if (rc) return rc;
            }
            HIPCHECK(c, launch_screen_est(ea, s));
        }
        ScreenArgs sa{};
        sa.U = c->d_U;
        sa.nshell = c->nshell;
        sa.nbatch = nb;
        sa.shell_l = c->d_shell_l;
        sa.shell_row = c->d_shell_row;
        sa.pairs = c->d_pairs;
        sa.eps_batch = eps_batch;
        sa.eps_low = eps_low;
        sa.nlist = c->nlist;
        sa.est = c->mlp ? c->d_est : nullptr;
        sa.thr = c->mlp ? c->d_thr : nullptr;
        sa.thr2 = c->mlp ? c->d_thr2 : nullptr;
        sa.ne_pos = c->d_ne_pos;
        sa.nne = (int64_t)c->ne_list.size();
        sa.counts = c->d_counts;
        sa.npairs = c->d_npairs;
        sa.skipped = c->d_skipped;
        sa.run_base = c->d_run_base;
        sa.bt_base = c->d_bt_base;
        const int ntile = (int)g.tiles.size();
        if (link) {
            HIPCHECK(c, launch_phisum(c->mixed ? nullptr : c->d_Phi, c->mixed ? c->d_Phi32 : nullptr, g.d_roff, ntile,
                                      c->tile_batches, g.tiles.back().ncols, c->d_pw + off, nb, c->d_phit, s));
            int rc = link_ftilde(c, g);
            if (rc) return rc;
            sa.link = 1;
            sa.link_eps = c->opts.eps_skip_energy;
            sa.fmax = c->d_fmax;
            sa.phit = c->d_phit;
            sa.atil = c->d_atil;
        }
        if (c->row_restrict) {
            HIPCHECK(c, launch_fill(c->d_shell_flag, (int64_t)ntile * c->nshell, 0, s));
            sa.shell_flag = c->d_shell_flag;
            sa.tile_batches = c->tile_batches;
        }
        if ((int)c->bound_order.size() == nb) {
            int rc = push_vector(c, c->bound_order, &sa.batch_order);   // the count pass only
            if (rc) return rc;
        }
        HIPCHECK(c, launch_screen(false, sa, s));
        const int NL = c->nlist;
        HIPCHECK(c, launch_screen_scan(c->d_counts, nb, NL, c->d_run_base, c->d_bt_base, s));
        if (c->row_restrict) {
            HIPCHECK(c, launch_tile_rows(c->d_shell_flag, ntile, c->nshell, c->d_shell_l, c->d_shell_row, c->nbf,
                                         c->d_trows, c->d_tcount, s));
            c->tile_rows.assign(ntile, 0);
            HIPCHECK(c, hipMemcpyAsync(c->tile_rows.data(), c->d_tcount, ntile * sizeof(int32_t),
                                       hipMemcpyDeviceToHost, s));
        }
        std::vector<int64_t> rb(NL * (size_t)(nb + 1)), bb(NL * (size_t)(nb + 1)), npair((size_t)nb * NL);
        std::vector<double> skipped(nb);
        HIPCHECK(c, hipMemcpyAsync(rb.data(), c->d_run_base, rb.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIPCHECK(c, hipMemcpyAsync(bb.data(), c->d_bt_base, bb.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIPCHECK(c, hipMemcpyAsync(npair.data(), c->d_npairs, npair.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIPCHECK(c, hipMemcpyAsync(skipped.data(), c->d_skipped, skipped.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHECK(c, hipStreamSynchronize(s));
        for (int k = 0; k < NL; ++k) {
            const int cl = k % 6;
            total_runs[k] = rb[(size_t)k * (nb + 1) + nb];
            int rc = ensure_pools(c, k, total_runs[k], bb[(size_t)k * (nb + 1) + nb]);
            if (rc) return rc;
            sa.runs[k] = c->d_pool_runs[k];
            sa.btasks[k] = c->d_pool_bt[k];
            sa.batch_run_off[k] = c->d_bro[k];
            const double avg_prims = c->ntask[cl] ? (double)c->task_prims[cl] / (double)c->ntask[cl] : 0.0;
            for (int j = 0; j < nb; ++j) {
                const int64_t u = npair[(size_t)j * NL + k] * npts[j];
                gs->pp[cl] += u;
                gs->ppp[cl] += (int64_t)(avg_prims * (double)u);
                if (k >= 6) gs->low += u;
            }
        }
        for (int j = 0; j < nb; ++j) gs->skipped += skipped[j];
        std::vector<uint8_t> key(nb);
        for (int k = 0; k < NL; ++k) {
            const int64_t* rk = &rb[(size_t)k * (nb + 1)];
            const int64_t* bk = &bb[(size_t)k * (nb + 1)];
            int32_t cnt[65] = {};   // batches per bucket: 64 = no runs, else 63 - floor(log2(B tasks + 1))
            for (int j = 0; j < nb; ++j) {
                const uint64_t n = (uint64_t)(bk[j + 1] - bk[j]) + 1;
                key[j] = rk[j + 1] > rk[j] ? (uint8_t)__builtin_clzll(n) : (uint8_t)64;
                ++cnt[key[j]];
            }
            const size_t first = order.size();
            order_off[k] = (int64_t)first;
            order_cnt[k] = nb - cnt[64];
            order.resize(first + order_cnt[k]);
            int32_t pos[64];
            for (int q = 0, p = 0; q < 64; ++q) {
                pos[q] = p;
                p += cnt[q];
            }
            for (int j = 0; j < nb; ++j)
                if (key[j] < 64) order[first + pos[key[j]]++] = j;
        }
        // the write pass of the lists: every batch (each writes its own records and offsets),
        // in decreasing powers of two of its B tasks over all lists.  (An uploaded record stays
        // valid only until the next upload, which may restart the staging arena: each order is
        // uploaded right before the launches that read it.)
        {
            std::vector<int32_t> worder(nb);
            int32_t cnt[64] = {};
            for (int j = 0; j < nb; ++j) {
                uint64_t n = 1;
                for (int k = 0; k < NL; ++k) n += (uint64_t)(bb[(size_t)k * (nb + 1) + j + 1] - bb[(size_t)k * (nb + 1) + j]);
                key[j] = (uint8_t)__builtin_clzll(n);
                ++cnt[key[j]];
            }
            int32_t pos[64];
            for (int q = 0, p = 0; q < 64; ++q) {
                pos[q] = p;
                p += cnt[q];
            }
            for (int j = 0; j < nb; ++j) worder[pos[key[j]]++] = j;
            int rc = push_vector(c, worder, &sa.batch_order);
            if (rc) return rc;
        }
        HIPCHECK(c, launch_screen(true, sa, s));
        if (c->kept_capture) {
            int rc = capture_kept(c, g, total_runs, bb);
            if (rc) return rc;
        }
        if (timed) HIPCHECK(c, hipEventRecord(c->ev[14], s));
    } else {
        for (int cl = 0; cl < 6; ++cl) {
            gs->pp[cl] += c->ntask[cl] * gpts;
            gs->ppp[cl] += c->task_prims[cl] * gpts;
            total_runs[cl] = c->nrun[cl];
        }
    }

    if (screen && c->row_restrict && !c->zero_f_rows && c->tile_rows.size() == g.tiles.size()) {
        // the A.F kernels update only the rows M_t of each tile's kept blocks: clear those, for
        // every tile in one launch
        std::vector<int64_t> cols(2 * g.tiles.size());
        int32_t max_rows = 0;
        for (size_t ti = 0; ti < g.tiles.size(); ++ti) {
            cols[2 * ti] = g.tiles[ti].col0;
            cols[2 * ti + 1] = g.tiles[ti].ncols;
            max_rows = std::max(max_rows, c->tile_rows[ti]);
        }
        const int64_t* d = nullptr;
        int rc = push_vector(c, cols, &d);
        if (rc) return rc;
        HIPCHECK(c, launch_fill_rows_tiles(c->d_G, ld, c->d_trows, nbf, c->d_tcount, d, (int32_t)g.tiles.size(),
                                           max_rows, 0.0, s));
    } else {
        HIPCHECK(c, launch_fill(c->d_G, nbf * g.ncols, 0.0, s));
    }
    AfgArgs a{};
    a.px = c->d_px + off;
    a.py = c->d_py + off;
    a.pz = c->d_pz + off;
    a.pw = c->d_pw + off;
    a.F = c->d_F;
    a.F32 = c->mixed ? c->d_F32 : nullptr;
    a.G = c->d_G;
    a.ld = ld;
    a.pairs = c->d_pairs;
    a.prims = c->d_prims;
    a.prims32 = c->d_prims32;
    a.rowc = c->d_rowc;
    a.nbatch = nb;
    a.boys_tab = c->d_boys;
    if (!order.empty()) {
        // the A.F launches' batch orders, uploaded after every other record of the group
        int rc = push_vector(c, order, &d_order);
        if (rc) return rc;
    }
    for (int cl = 0; cl < 6; ++cl) {
        if (timed) HIPCHECK(c, hipEventRecord(c->ev[8 + cl], s));
        // the class's FP64 list, then (mixed build) its FP32 list
        for (int k = cl; k < (screen ? c->nlist : 6); k += 6) {
            if (total_runs[k] == 0) continue;
            if (screen) {
                a.runs = c->d_pool_runs[k];
                a.btasks = c->d_pool_bt[k];
                a.batch_run_off = c->d_bro[k];
                a.nrun = 0;
                a.batch_order = d_order + order_off[k];
                a.nbatch = order_cnt[k];
            } else {
                a.runs = c->d_runs[cl];
                a.btasks = c->d_btasks[cl];
                a.batch_run_off = nullptr;
                a.nrun = c->nrun[cl];
                a.batch_order = nullptr;
                a.nbatch = nb;
            }
            a.lowp = k >= 6;
            HIPCHECK(c, launch_afg(kClassLA[cl], kClassLB[cl], a, s));
        }
        if (timed) HIPCHECK(c, hipEventRecord(c->ev[cl == 5 ? 15 : 9 + cl], s));
    }
    if (timed) HIPCHECK(c, hipEventRecord(c->ev[3], s));
    return SNK_OK;
}

}  // namespace

namespace {

// Points the context's stream and group buffers at pipeline set k for the
// duration of a build, and back to the context's own at restore() or destruction.
struct PipeSwap {
    snk_ctx* c;
    bool on;
    hipStream_t s0;
    PipeSwap(snk_ctx* x, bool active) : c(x), on(active), s0(x->stream) {}
    void use(int k)
    {
        c->stream = c->pstream[k];
        c->d_Phi = c->p_Phi[k];
        c->d_F = c->p_F[k];
        c->d_G = c->p_G[k];
        c->d_part = c->p_part[k];
    }
    void restore()
    {
        if (!on) return;
        c->stream = s0;
        c->d_Phi = c->p_Phi[0];
        c->d_F = c->p_F[0];
        c->d_G = c->p_G[0];
        c->d_part = c->p_part[0];
        on = false;
    }
    ~PipeSwap() { restore(); }
};

}  // namespace

namespace {

// Host-pointer density matrix: finite elements, and with SNK_VALIDATE symmetric to
// 1e-12 of its largest element.
int check_density(snk_ctx* c, const double* P)
{
    const int64_t nbf = c->nbf;
    const size_t nb2 = (size_t)nbf * nbf;
    for (size_t k = 0; k < nb2; ++k)
        if (!isfin(P[k])) return arg_error(c, "non-finite density matrix element");
    if (c->opts.flags & SNK_VALIDATE) {
        double mx = 0.0, asym = 0.0;
        for (int64_t i = 0; i < nbf; ++i)
            for (int64_t j = 0; j < nbf; ++j) {
                mx = std::max(mx, std::fabs(P[i * nbf + j]));
                asym = std::max(asym, std::fabs(P[i * nbf + j] - P[j * nbf + i]));
            }
        if (asym > 1e-12 * mx) {
            set_err(c, "density matrix is not symmetric");
            return SNK_E_ASYM;
        }
    }
    return SNK_OK;
}

// XC workspace: chunks of whole batches sized to the device budget (three nbf-row buffers of
// FP64 per column: Phi, F, G), and the split of the Z Phi^T product over grid points that fills the
// device with nbf x nbf outputs of 64 x 64 tiles.
int xc_workspace(snk_ctx* c)
{
    const int64_t nbf = c->nbf;
    const int64_t total = (int64_t)c->nbatch * kBatch;
    int64_t budget = c->opts.max_device_bytes;
    if (budget <= 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = (size_t)8 << 30;
        budget = (int64_t)(0.25 * (double)fr);
    }
    // split partial products of the V product: at most half the budget
    c->xc_nsplit = (int)std::max<int64_t>(
        1, std::min<int64_t>(choose_ksplit(out_tiles(nbf, nbf), 256), budget / 2 / std::max<int64_t>(1, nbf * nbf * 8)));
    budget -= (int64_t)c->xc_nsplit * nbf * nbf * 8;
    const int64_t per_col = 3 * nbf * 8 + 16;
    int64_t cols = budget / per_col;
    cols = std::min<int64_t>(total, cols - cols % kBatch);
    if (cols < kBatch) {
        set_err(c, "device budget smaller than one batch of the XC workspace");
        return SNK_E_NOMEM;
    }
    c->xc_cols = cols;
    // one point-kernel tile per chunk: every shell, F and G rows of stride ncols from 0
    std::vector<XcTile> tiles;
    for (int64_t col0 = 0; col0 < total; col0 += cols)
        tiles.push_back(XcTile{0, (int32_t)std::min<int64_t>(cols, total - col0), 0, c->nshell, 0});
    std::vector<int32_t> shells((size_t)c->nshell);
    std::iota(shells.begin(), shells.end(), 0);
    int rc = 0;
    if ((rc = dalloc(c, &c->d_xphi, (size_t)(nbf * cols))) || (rc = dalloc(c, &c->d_xF, (size_t)(nbf * cols))) ||
        (rc = dalloc(c, &c->d_xG, (size_t)(nbf * cols))) || (rc = dalloc(c, &c->d_xe, (size_t)(2 * cols))) ||
        (rc = dalloc(c, &c->d_xred, 512)) || (rc = upload(c, &c->d_xtiles, tiles)) ||
        (rc = upload(c, &c->d_xshells, shells)) || (rc = dalloc(c, &c->d_xsum, 2))) {
        for (double** p : {&c->d_xphi, &c->d_xF, &c->d_xG, &c->d_xe, &c->d_xred, &c->d_xsum}) {
            (void)hipFree(*p);
            *p = nullptr;
        }
        (void)hipFree(c->d_xtiles);
        (void)hipFree(c->d_xshells);
        c->d_xtiles = nullptr;
        c->d_xshells = nullptr;
        return rc;
    }
    return SNK_OK;
}

// Basis-screened XC (eps_basis > 0): one batch group at a time in the sn-K group layout
// (tile t's Phi_t, F_t and G_t at phi_off, |B_t| rows of stride ncols_t), one point-kernel
// launch per group, the tile products one after the other.
int xc_workspace_tiled(snk_ctx* c)
{
    int64_t cols = kBatch;
    std::vector<XcTile> tiles;
    std::vector<int32_t> shells;
    c->xc_gt0.clear();
    for (const Group& g : c->groups) {
        cols = std::max<int64_t>(cols, g.ncols);
        c->xc_gt0.push_back((int32_t)tiles.size());
        for (const Tile& t : g.tiles) {
            tiles.push_back(XcTile{t.phi_off, (int32_t)t.ncols, (int32_t)shells.size(), (int32_t)t.coll_shells.size(), 0});
            shells.insert(shells.end(), t.coll_shells.begin(), t.coll_shells.end());
        }
    }
    const int64_t elems = std::max<int64_t>(1, c->max_phi);
    c->xc_cols = cols;
    c->xc_nsplit = kBasisTileBatches;
    int rc = 0;
    if ((rc = dalloc(c, &c->d_xphi, (size_t)elems)) || (rc = dalloc(c, &c->d_xF, (size_t)elems)) ||
        (rc = dalloc(c, &c->d_xG, (size_t)elems)) || (rc = dalloc(c, &c->d_xe, (size_t)(2 * cols))) ||
        (rc = dalloc(c, &c->d_xred, 512)) || (rc = upload(c, &c->d_xtiles, tiles)) ||
        (rc = upload(c, &c->d_xshells, shells)) || (rc = dalloc(c, &c->d_xsum, 2))) {
        for (double** p : {&c->d_xphi, &c->d_xF, &c->d_xG, &c->d_xe, &c->d_xred, &c->d_xsum}) {
            (void)hipFree(*p);
            *p = nullptr;
        }
        (void)hipFree(c->d_xtiles);
        (void)hipFree(c->d_xshells);
        c->d_xtiles = nullptr;
        c->d_xshells = nullptr;
        return rc;
    }
    return SNK_OK;
}

// One batch group of the basis-screened XC build: Phi_t over B_t per tile, F_t = P[B_t, B_t] Phi_t
// for every tile in one grouped launch (P read in place), the point kernel over all tiles at
// once, then Kt[B_t, B_t] += G_t Phi_t^T for every tile in one grouped launch (split per
// batch) and one fixed-order reduction of all tiles into Kt.
int xc_group(snk_ctx* c, size_t gi, const double* dP, int functional)
{
    hipStream_t s = c->stream;
    const Group& g = c->groups[gi];
    const int64_t nbf = c->nbf, goff = (int64_t)g.b0 * kBatch;
    const int ntile = (int)g.tiles.size();
    std::vector<GemmProb> fp, vp;
    std::vector<RedTile> red;
    int64_t need = 0;
    for (const Tile& t : g.tiles) need += (int64_t)(t.b1 - t.b0) * t.nB * t.nB;
    int rc = ensure_part(c, need);
    if (rc) return rc;
    int64_t poff = 0;
    int32_t max_nb = 0;
    for (int ti = 0; ti < ntile; ++ti) {
        const Tile& t = g.tiles[ti];
        if (t.nB == 0) continue;
        max_nb = std::max(max_nb, t.nB);
        const int64_t ncols = t.ncols, off = (int64_t)t.b0 * kBatch;
        HIPCHECK(c, launch_collocate(c->d_px + off, c->d_py + off, c->d_pz + off, ncols, c->d_shells, c->d_exps,
                                     c->d_coefs, t.d_coll_shells, t.d_coll_rows, (int32_t)t.coll_shells.size(),
                                     c->d_xphi + t.phi_off, ncols, s));
        GemmProb p{};
        p.A = dP;
        p.lda = nbf;
        p.arow = t.d_coll_fn;
        p.acol = t.d_coll_fn;
        p.B = c->d_xphi + t.phi_off;
        p.ldb = ncols;
        p.C = c->d_xF + t.phi_off;
        p.ldc = ncols;
        p.M = t.nB;
        p.N = (int32_t)ncols;
        p.K = t.nB;
        p.ksplit = 1;
        fp.push_back(p);
        GemmProb v{};
        v.A = c->d_xG + t.phi_off;
        v.lda = ncols;
        v.B = c->d_xphi + t.phi_off;
        v.ldb = ncols;
        v.C = c->d_part + poff;
        v.ldc = t.nB;
        v.cstride = (int64_t)t.nB * t.nB;
        v.M = t.nB;
        v.N = t.nB;
        v.K = (int32_t)ncols;
        v.ksplit = t.b1 - t.b0;
        vp.push_back(v);
        RedTile r{};
        r.poff = poff;
        r.M = t.nB;
        r.N = t.nB;
        r.ksplit = v.ksplit;
        r.rinv = c->d_rinv + (int64_t)ti * nbf;
        r.ccol = t.d_coll_fn;
        red.push_back(r);
        poff += (int64_t)v.ksplit * t.nB * t.nB;
    }
    if ((rc = run_gemms(c, fp, kGemmF64, false))) return rc;
    HIPCHECK(c, launch_xc_point(c->d_px + goff, c->d_py + goff, c->d_pz + goff, c->d_pw + goff, g.ncols, c->d_shells,
                                c->d_exps, c->d_coefs, c->d_xtiles + c->xc_gt0[gi], c->d_xshells, c->tile_batches,
                                c->d_xF, functional, c->d_xG, c->d_xe, s));
    HIPCHECK(c, launch_xc_sum(c->d_xe, g.ncols, c->d_xred, c->d_xsum, true, s));
    if ((rc = run_gemms(c, vp, kGemmF64, true))) return rc;
    HIPCHECK(c, launch_rinv(g.d_fn_cat, 0, g.d_roff, nullptr, ntile, nbf, max_nb, c->d_rinv, s));
    return run_reduce(c, red, c->d_Kt);
}

// Combined build: workspace of the group-sized XC buffers (FP64 contexts without basis
// screening, one tile per group spanning every function).
int kx_workspace(snk_ctx* c)
{
    const int64_t nbf = c->nbf, cols = std::max<int64_t>(kBatch, c->max_cols);
    c->kx_nsplit = choose_ksplit(out_tiles(nbf, nbf), 256);
    std::vector<XcTile> tiles;
    for (const Group& g : c->groups) tiles.push_back(XcTile{0, (int32_t)g.ncols, 0, c->nshell, 0});
    std::vector<int32_t> shells((size_t)c->nshell);
    std::iota(shells.begin(), shells.end(), 0);
    int rc = 0;
    if ((rc = dalloc(c, &c->d_kxe, (size_t)(2 * cols))) ||
        (rc = dalloc(c, &c->d_kxKt, (size_t)(nbf * nbf))) || (rc = dalloc(c, &c->d_kxred, 512)) ||
        (rc = upload(c, &c->d_kxtiles, tiles)) || (rc = upload(c, &c->d_kxshells, shells)) ||
        (rc = dalloc(c, &c->d_kxsum, 3))) {
        for (double** p : {&c->d_kxe, &c->d_kxKt, &c->d_kxred, &c->d_kxsum}) {
            (void)hipFree(*p);
            *p = nullptr;
        }
        (void)hipFree(c->d_kxtiles);
        (void)hipFree(c->d_kxshells);
        c->d_kxtiles = nullptr;
        c->d_kxshells = nullptr;
        return rc;
    }
    return SNK_OK;
}

// Eq. vxc_num over ncols points of every function: T += G Phi^T (G and Phi nbf x ncols), split
// over ksplit chunks of points and reduced in a fixed order
int xc_vproduct(snk_ctx* c, const double* G, const double* Phi, int64_t ncols, int ksplit, double* T)
{
    const int64_t nbf = c->nbf;
    ksplit = std::max(1, ksplit);
    int rc = ensure_part(c, (int64_t)ksplit * nbf * nbf);
    if (rc) return rc;
    std::vector<GemmProb> vp(1);
    GemmProb& v = vp[0];
    v = GemmProb{};
    v.A = G;
    v.lda = ncols;
    v.B = Phi;
    v.ldb = ncols;
    v.C = c->d_part;
    v.ldc = nbf;
    v.cstride = nbf * nbf;
    v.M = (int32_t)nbf;
    v.N = (int32_t)nbf;
    v.K = (int32_t)ncols;
    v.ksplit = ksplit;
    if ((rc = run_gemms(c, vp, kGemmF64, true))) return rc;
    std::vector<RedTile> red(1);
    red[0] = RedTile{};
    red[0].M = (int32_t)nbf;
    red[0].N = (int32_t)nbf;
    red[0].ksplit = ksplit;
    return run_reduce(c, red, T);
}

// Combined build, group gi: the XC point kernel on the group's Phi and F (Eqs. den_grid,
// exc_grid, zmat) and Kt_xc += G_xc Phi^T (Eq. vxc_num), on the context's stream after the
// group's K product, before the next group reuses Phi and F.  G_xc = 2 Z takes the place of
// the exchange G, which the K product has consumed by then.
int group_kx(snk_ctx* c, size_t gi)
{
    hipStream_t s = c->stream;
    const Group& g = c->groups[gi];
    const int64_t nbf = c->nbf, ncols = g.ncols, off = (int64_t)g.b0 * kBatch;
    const double* Phi = c->d_Phi + g.tiles[0].phi_off;
    HIPCHECK(c, launch_xc_point(c->d_px + off, c->d_py + off, c->d_pz + off, c->d_pw + off, ncols, c->d_shells,
                                c->d_exps, c->d_coefs, c->d_kxtiles + gi, c->d_kxshells, (int32_t)(ncols / kBatch),
                                c->d_F, c->kx_fn, c->d_G, c->d_kxe, s));
    HIPCHECK(c, launch_xc_sum(c->d_kxe, ncols, c->d_kxred, c->d_kxsum, true, s));
    return xc_vproduct(c, c->d_G, Phi, ncols, std::min<int>(c->kx_nsplit, (int)(ncols / kBatch)), c->d_kxKt);
}

}  // namespace

extern "C" {

int snk_vxc_build(snk_ctx* c, const double* P, int functional, double* V_out, double* exc_out, double* nel_out)
{
    if (!c) return arg_error(nullptr, "context is NULL");
    if (!P || !V_out) return arg_error(c, "P or V_out is NULL");
    if (functional < SNK_XC_SLATER || functional > SNK_XC_PBE) return arg_error(c, "unknown functional");
    const bool dev = (c->opts.flags & SNK_DEVICE_PTRS) != 0;
    const int64_t nbf = c->nbf;
    const size_t nb2 = (size_t)nbf * nbf;
    if (!dev) {
        int rc = check_density(c, P);
        if (rc) return rc;
    }
    HIPCHECK(c, hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const double* dP = P;
    double* dV = V_out;
    if (!dev) {
        HIPCHECK(c, hipMemcpyAsync(c->d_P, P, nb2 * sizeof(double), hipMemcpyHostToDevice, s));
        dP = c->d_P;
        dV = c->d_K;
    }
    const int64_t total = (int64_t)c->nbatch * kBatch;
    const bool tiled = c->opts.eps_basis > 0.0;
    if (!c->d_xsum) {
        int rc = total > 0 && nbf > 0 ? (tiled ? xc_workspace_tiled(c) : xc_workspace(c)) : dalloc(c, &c->d_xsum, 2);
        if (rc) return rc;
    }
    HIPCHECK(c, launch_fill(c->d_Kt, (int64_t)nb2, 0.0, s));
    HIPCHECK(c, launch_fill(c->d_xsum, 2, 0.0, s));
    if (tiled && total > 0) {
        for (size_t gi = 0; gi < c->groups.size(); ++gi) {
            int rc = xc_group(c, gi, dP, functional);
            if (rc) return rc;
        }
    }
    for (int64_t col0 = 0, chunk = 0; col0 < total && nbf > 0 && !tiled; col0 += c->xc_cols, ++chunk) {
        const int64_t ncols = std::min<int64_t>(c->xc_cols, total - col0);
        // Eqs. collocation, fmat
        HIPCHECK(c, launch_xc_collocate(c->d_px + col0, c->d_py + col0, c->d_pz + col0, ncols, c->d_shells, c->d_exps,
                                        c->d_coefs, c->d_shell_row, c->nshell, c->d_xphi, s));
        {
            std::vector<GemmProb> fp(1);
            fp[0] = GemmProb{};
            fp[0].A = dP;
            fp[0].lda = nbf;
            fp[0].B = c->d_xphi;
            fp[0].ldb = ncols;
            fp[0].C = c->d_xF;
            fp[0].ldc = ncols;
            fp[0].M = (int32_t)nbf;
            fp[0].N = (int32_t)ncols;
            fp[0].K = (int32_t)nbf;
            fp[0].ksplit = 1;
            int rc = run_gemms(c, fp, kGemmF64, false);
            if (rc) return rc;
        }
        // Eqs. den_grid, exc_grid, zmat
        HIPCHECK(c, launch_xc_point(c->d_px + col0, c->d_py + col0, c->d_pz + col0, c->d_pw + col0, ncols, c->d_shells,
                                    c->d_exps, c->d_coefs, c->d_xtiles + chunk, c->d_xshells,
                                    (int32_t)(ncols / kBatch), c->d_xF, functional, c->d_xG, c->d_xe, s));
        HIPCHECK(c, launch_xc_sum(c->d_xe, ncols, c->d_xred, c->d_xsum, true, s));
        // Eq. vxc_num: Kt += G Phi^T over the chunk's points, split over points, fixed-order sum
        int rc = xc_vproduct(c, c->d_xG, c->d_xphi, ncols, std::min<int>(c->xc_nsplit, (int)(ncols / kBatch)), c->d_Kt);
        if (rc) return rc;
    }
    // V = (Kt + Kt^T) / 2 with G = 2 Z; the finish's trace term is not used here
    HIPCHECK(c, launch_finish(c->d_Kt, dP, dV, nbf, c->d_partial, c->nfinish, c->d_ex, s));
    double sums[2] = {0.0, 0.0};
    if (!dev) HIPCHECK(c, hipMemcpyAsync(V_out, dV, nb2 * sizeof(double), hipMemcpyDeviceToHost, s));
    if (!dev || exc_out || nel_out) {
        HIPCHECK(c, hipMemcpyAsync(sums, c->d_xsum, sizeof(sums), hipMemcpyDeviceToHost, s));
        HIPCHECK(c, hipStreamSynchronize(s));
    }
    if (exc_out) *exc_out = sums[0];
    if (nel_out) *nel_out = sums[1];
    return SNK_OK;
}

int snk_ctx_build_kxc(snk_ctx* c, const double* P, double* K_out, int functional, double* V_out, double* exc_out,
                      double* nel_out, snk_stats* stats)
{
    if (!c) return arg_error(nullptr, "context is NULL");
    if (!P || !K_out || !V_out) return arg_error(c, "P, K_out or V_out is NULL");
    if (functional < SNK_XC_SLATER || functional > SNK_XC_PBE) return arg_error(c, "unknown functional");
    const bool share = !c->mixed && c->opts.eps_basis <= 0.0 && !c->pipe && c->nbatch > 0 && c->nbf > 0;
    if (!share) {
        int rc = snk_ctx_build(c, P, K_out, stats);
        return rc ? rc : snk_vxc_build(c, P, functional, V_out, exc_out, nel_out);
    }
    HIPCHECK(c, hipSetDevice(c->device));
    if (!c->d_kxsum) {
        int rc = kx_workspace(c);
        if (rc) return rc;
    }
    const bool dev = (c->opts.flags & SNK_DEVICE_PTRS) != 0;
    const size_t nb2 = (size_t)c->nbf * c->nbf;
    c->kx_fn = functional;
    int rc = snk_ctx_build(c, P, K_out, stats);
    c->kx_fn = 0;
    if (rc) return rc;
    hipStream_t s = c->stream;
    const double* dP = dev ? P : c->d_P;     // uploaded by the sn-K build in host-pointer mode
    double* dV = dev ? V_out : c->d_K;
    // V = (Kt_xc + Kt_xc^T) / 2 with G = 2 Z (Eq. vxc_num); the trace goes to an unused slot
    HIPCHECK(c, launch_finish(c->d_kxKt, dP, dV, c->nbf, c->d_partial, c->nfinish, c->d_kxsum + 2, s));
    double sums[2] = {0.0, 0.0};
    if (!dev) HIPCHECK(c, hipMemcpyAsync(V_out, dV, nb2 * sizeof(double), hipMemcpyDeviceToHost, s));
    if (!dev || exc_out || nel_out) {
        HIPCHECK(c, hipMemcpyAsync(sums, c->d_kxsum, sizeof(sums), hipMemcpyDeviceToHost, s));
        HIPCHECK(c, hipStreamSynchronize(s));
    }
    if (exc_out) *exc_out = sums[0];
    if (nel_out) *nel_out = sums[1];
    return SNK_OK;
}

int snk_ctx_build(snk_ctx* c, const double* P, double* K_out, snk_stats* stats)
{
    if (!c) return arg_error(nullptr, "context is NULL");
    if (!P || !K_out) return arg_error(c, "P or K_out is NULL");
    const bool dev = (c->opts.flags & SNK_DEVICE_PTRS) != 0;
    const int64_t nbf = c->nbf;
    const size_t nb2 = (size_t)nbf * nbf;
    if (!dev) {
        int rc = check_density(c, P);
        if (rc) return rc;
    }
    const auto t_start = std::chrono::steady_clock::now();
    HIPCHECK(c, hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const double* dP = P;
    double* dK = K_out;
    if (!dev) {
        HIPCHECK(c, hipMemcpyAsync(c->d_P, P, nb2 * sizeof(double), hipMemcpyHostToDevice, s));
        dP = c->d_P;
        dK = c->d_K;
    }
    double tcol = 0, tf = 0, tafg = 0, tk = 0, tscr = 0;
    c->acc_fn = c->acc_frows = c->acc_grows = c->acc_cols = 0.0;
    double tcls[6] = {0, 0, 0, 0, 0, 0};
    GroupStats gs;
    const bool timed = stats != nullptr;
    c->timing = timed;
    for (int k = 0; k < 4; ++k) {
        c->gms[k] = 0.0;
        c->gcount[k] = 0;
    }

    HIPCHECK(c, launch_fill(c->d_Kt, (int64_t)nb2, 0.0, s));
    c->d_P_cur = dP;
    c->acc_flops64 = c->acc_flops32 = 0.0;
    for (auto& f : c->slot_flops) f[0] = f[1] = 0.0;
    if (c->split) HIPCHECK(c, launch_fill(c->d_lpb + (int64_t)c->max_group_tiles * kBoundChunksPerTile, 1, 0.0, s));
    if (c->kx_fn) {
        HIPCHECK(c, launch_fill(c->d_kxKt, (int64_t)nb2, 0.0, s));
        HIPCHECK(c, launch_fill(c->d_kxsum, 3, 0.0, s));
    }
    if (c->mixed) HIPCHECK(c, launch_convert_f32(dP, (int64_t)nb2, c->d_P32, s));
    {
        int rc = link_prepare(c, dP);
        if (rc) return rc;
    }
    if (c->mlp)
        HIPCHECK(c, launch_pair_pnorm(dP, nbf, c->d_ne_list, c->d_pa, c->d_pb, c->d_shell_l, c->d_shell_row,
                                      (int64_t)c->ne_list.size(), c->d_lp, s));
    // two groups at once (untimed plain FP64 builds): group gi runs on pipeline stream gi % 2
    // with buffer set gi % 2; its reductions into Kt wait for those of group gi - 1
    const bool pipe = c->pipe && c->groups.size() > 1 && !timed;
    PipeSwap swap(c, pipe);
    if (pipe) {
        HIPCHECK(c, hipEventRecord(c->pev_fork, s));
        for (int k = 0; k < 2; ++k) HIPCHECK(c, hipStreamWaitEvent(c->pstream[k], c->pev_fork, 0));
    }
    for (size_t gi = 0; gi < c->groups.size(); ++gi) {
        const Group& g = c->groups[gi];
        if (pipe) swap.use((int)(gi & 1));
        int rc = group_until_G(c, g, dP, timed, &gs);
        if (rc) return rc;
        if (pipe && gi > 0) HIPCHECK(c, hipStreamWaitEvent(c->stream, c->pev_k[(gi - 1) & 1], 0));
        if ((rc = group_K(c, g))) return rc;
        if (pipe) HIPCHECK(c, hipEventRecord(c->pev_k[gi & 1], c->stream));
        if (timed) {
            HIPCHECK(c, hipEventRecord(c->ev[4], s));
            HIPCHECK(c, hipEventSynchronize(c->ev[4]));
            for (int k = 0; k < 4; ++k)
                if (c->gl[k]) {
                    c->gms[k] += ev_ms(c->gev[2 * k], c->gev[2 * k + 1]);
                    c->gcount[k] += 1;
                    c->gl[k] = false;
                }
            tcol += ev_ms(c->ev[0], c->ev[1]);
            tf += ev_ms(c->ev[1], c->ev[2]);
            if (c->opts.screen != SNK_SCREEN_NONE) {
                tscr += ev_ms(c->ev[7], c->ev[14]);
                tafg += ev_ms(c->ev[14], c->ev[3]);
            } else {
                tafg += ev_ms(c->ev[2], c->ev[3]);
            }
            for (int cl = 0; cl < 6; ++cl) {
                if (gs.pp[cl] == 0) continue;
                tcls[cl] += ev_ms(c->ev[8 + cl], c->ev[cl == 5 ? 15 : 9 + cl]);
            }
            tk += ev_ms(c->ev[3], c->ev[4]);
        }
        // combined build: the XC potential from this group's Phi and F (outside the sn-K phase timings)
        if (c->kx_fn && (rc = group_kx(c, gi))) return rc;
    }
    if (pipe) {
        swap.restore();
        for (int k = 0; k < 2; ++k) {
            HIPCHECK(c, hipEventRecord(c->pev_end[k], c->pstream[k]));
            HIPCHECK(c, hipStreamWaitEvent(s, c->pev_end[k], 0));
        }
    }
    // Eq. sn_k and E_x
    if (timed) HIPCHECK(c, hipEventRecord(c->ev[5], s));
    HIPCHECK(c, launch_finish(c->d_Kt, dP, dK, nbf, c->d_partial, c->nfinish, c->d_ex, s));
    if (timed) HIPCHECK(c, hipEventRecord(c->ev[6], s));
    double ex = 0.0;
    if (!dev) {
        HIPCHECK(c, hipMemcpyAsync(K_out, dK, nb2 * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    if (!dev || timed) {
        HIPCHECK(c, hipMemcpyAsync(&ex, c->d_ex, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHECK(c, hipStreamSynchronize(s));
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->ex = ex;
        stats->t_total_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        stats->t_collocate_ms = tcol;
        stats->t_fgemm_ms = tf;
        stats->t_afg_ms = tafg;
        stats->t_kgemm_ms = tk;
        stats->t_finish_ms = ev_ms(c->ev[5], c->ev[6]);
        int64_t evaluated = 0;
        for (int k = 0; k < 6; ++k) {
            stats->pair_points[k] = gs.pp[k];
            stats->prim_pair_points[k] = gs.ppp[k];
            stats->t_afg_class_ms[k] = tcls[k];
            evaluated += gs.pp[k];
        }
        stats->t_screen_ms = tscr;
        stats->pair_points_skipped = gs.cand - evaluated;
        stats->pair_points_lowprec = gs.low;
        stats->skipped_bound = gs.skipped;
        stats->n_batches = c->nbatch;
        stats->n_groups = (int32_t)c->groups.size();
        const double cols = std::max(1.0, c->acc_cols);
        stats->tile_functions = c->acc_fn / cols;
        stats->tile_frows = c->acc_frows / cols;
        stats->tile_grows = c->row_restrict ? c->acc_grows / cols : (double)nbf;
        stats->gemm_flops_fp64 = c->acc_flops64;
        stats->gemm_flops_fp32 = c->acc_flops32;
        for (int k = 0; k < 4; ++k) {
            stats->t_gemm_ms[k] = c->gms[k];
            stats->gemm_launches[k] = c->gcount[k];
            stats->gemm_kind_flops[k][0] = c->slot_flops[k][0];
            stats->gemm_kind_flops[k][1] = c->slot_flops[k][1];
        }
        if (c->split) {
            double sum = 0.0;
            HIPCHECK(c, hipMemcpy(&sum, c->d_lpb + (int64_t)c->max_group_tiles * kBoundChunksPerTile, sizeof(double),
                                  hipMemcpyDeviceToHost));
            stats->lowprec_bound = kFp32GemmGamma * kWeakPhi * sum;
        }
    }
    return SNK_OK;
}

int sn_k_build(const snk_basis* basis, const snk_grid* grid, const double* weights, const double* P, double* K_out,
               const snk_opts* opts)
{
    if (!P || !K_out) return arg_error(nullptr, "P or K_out is NULL");
    snk_ctx* c = nullptr;
    int rc = snk_ctx_create(basis, grid, weights, opts, &c);
    if (rc) return rc;
    rc = snk_ctx_build(c, P, K_out, opts ? opts->stats : nullptr);
    if (rc) g_last_error = c->err;
    snk_ctx_destroy(c);
    return rc;
}

int snk_shell_rcut(int l, const double* exps, const double* coefs, int nprim, double eps, double* r_out)
{
    if (!exps || !coefs || !r_out) return arg_error(nullptr, "NULL argument");
    if (l < 0 || l > kMaxL || nprim < 1 || !isfin(eps) || eps <= 0.0) return arg_error(nullptr, "bad shell or eps");
    for (int k = 0; k < nprim; ++k)
        if (!isfin(exps[k]) || exps[k] <= 0.0 || !isfin(coefs[k])) return arg_error(nullptr, "bad exponent or coefficient");
    *r_out = shell_rcut(l, exps, coefs, nprim, eps);
    return SNK_OK;
}

int snk_debug_gemm_f64(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* B, int64_t ldb,
                       int bt, double* C, int64_t ldc, int tile, void* stream)
{
    if (M < 0 || N < 0 || K < 0 || !A || !B || !C) return arg_error(nullptr, "bad GEMM arguments");
    if (tile != 0 && tile != kTile64 && tile != kTile128 && tile != kTile64x128 && tile != kTile128x256)
        return arg_error(nullptr, "tile must be 0, 64, 128, 192 or 384");
    if (M == 0 || N == 0) return SNK_OK;
    if (lda < K || ldc < N || ldb < (bt ? K : N)) return arg_error(nullptr, "leading dimension too small");
    if (M > INT32_MAX || N > INT32_MAX || K > INT32_MAX) return arg_error(nullptr, "GEMM too large");
    GemmProb p{};
    p.A = A;
    p.lda = lda;
    p.B = B;
    p.ldb = ldb;
    p.C = C;
    p.ldc = ldc;
    p.M = (int32_t)M;
    p.N = (int32_t)N;
    p.K = (int32_t)K;
    p.ksplit = 1;
    if (tile == 0) tile = ggemm_tile(&p, 1);
    ggemm_plan(p, tile, 8, 8);
    GemmProb* d = nullptr;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMalloc((void**)&d, sizeof(GemmProb));
    if (e == hipSuccess) e = hipMemcpyAsync(d, &p, sizeof(GemmProb), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_ggemm_f64(d, 1, ggemm_workgroups(p), tile, bt != 0, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d);
    if (e != hipSuccess) {
        g_last_error = hipGetErrorString(e);
        return SNK_E_DEVICE;
    }
    return SNK_OK;
}

int snk_debug_frow_prefilter(int on)
{
    if (on != 0 && on != 1) return arg_error(nullptr, "on must be 0 or 1");
    g_frow_prefilter = on;
    return SNK_OK;
}

int snk_debug_force_tile(int tile)
{
    if (tile != 0 && tile != kTile64 && tile != kTile128 && tile != kTile64x128 && tile != kTile128x256)
        return arg_error(nullptr, "tile must be 0, 64, 128, 192 or 384");
    g_force_tile = tile;
    return SNK_OK;
}

int snk_debug_mfma_layout(double* out)
{
    if (!out) return arg_error(nullptr, "NULL output");
    double* d = nullptr;
    if (hipMalloc((void**)&d, 256 * sizeof(double)) != hipSuccess) return SNK_E_NOMEM;
    hipError_t e = launch_mfma_probe(d, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out, d, 256 * sizeof(double), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) {
        g_last_error = hipGetErrorString(e);
        return SNK_E_DEVICE;
    }
    return SNK_OK;
}

int snk_ctx_point_order(const snk_ctx* c, int64_t* col_to_point)
{
    if (!c || !col_to_point) return arg_error(nullptr, "NULL argument");
    std::copy(c->col_point.begin(), c->col_point.end(), col_to_point);
    return SNK_OK;
}

// Sets snk_ctx::zero_f_rows for the lifetime of a call that reads every row of F or G.
struct ZeroRows {
    snk_ctx* c;
    explicit ZeroRows(snk_ctx* x) : c(x) { c->zero_f_rows = true; }
    ~ZeroRows() { c->zero_f_rows = false; }
};

int snk_ctx_debug_intermediates(snk_ctx* c, const double* P, double* Phi, double* F, double* G, int64_t* ncols_out)
{
    if (!c || !P) return arg_error(c, "NULL argument");
    ZeroRows zr(c);
    if (c->mixed) return arg_error(c, "intermediates are available from FP64 contexts only");
    if (c->groups.empty()) {
        if (ncols_out) *ncols_out = 0;
        return SNK_OK;
    }
    const Group& g = c->groups[0];
    const int64_t nbf = c->nbf;
    HIPCHECK(c, hipSetDevice(c->device));
    HIPCHECK(c, hipMemcpyAsync(c->d_P, P, (size_t)nbf * nbf * sizeof(double), hipMemcpyHostToDevice, c->stream));
    GroupStats gs;
    int rc = link_prepare(c, c->d_P);
    if (rc) return rc;
    rc = group_until_G(c, g, c->d_P, false, &gs);
    if (rc) return rc;
    const size_t n = (size_t)nbf * g.ncols * sizeof(double);
    std::vector<double> phig(Phi ? (size_t)g.phi_elems : 0);
    if (!phig.empty())
        HIPCHECK(c, hipMemcpyAsync(phig.data(), c->d_Phi, phig.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (F) HIPCHECK(c, hipMemcpyAsync(F, c->d_F, n, hipMemcpyDeviceToHost, c->stream));
    if (G) HIPCHECK(c, hipMemcpyAsync(G, c->d_G, n, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    if (Phi) {
        // elements of functions outside a tile's B_t are zero
        std::fill(Phi, Phi + (size_t)nbf * g.ncols, 0.0);
        for (const Tile& t : g.tiles)
            for (int32_t r = 0; r < t.nB; ++r) {
                const auto src = phig.begin() + t.phi_off + (int64_t)r * t.ncols;
                std::copy(src, src + t.ncols, Phi + (size_t)t.coll_fn[r] * g.ncols + t.col0);
            }
    }
    if (ncols_out) *ncols_out = g.ncols;
    return SNK_OK;
}

int64_t snk_ctx_nblock_pairs(const snk_ctx* c) { return c ? (int64_t)c->ne_list.size() : 0; }

int snk_ctx_ngroups(const snk_ctx* c) { return c ? (int)c->groups.size() : 0; }

int snk_ctx_ntiles(const snk_ctx* c)
{
    int n = 0;
    if (c)
        for (const Group& g : c->groups) n += (int)g.tiles.size();
    return n;
}

int snk_ctx_tile_info(const snk_ctx* c, int32_t* group, int32_t* b0, int32_t* b1, int32_t* nB)
{
    if (!c) return arg_error(nullptr, "context is NULL");
    size_t k = 0;
    for (size_t gi = 0; gi < c->groups.size(); ++gi)
        for (const Tile& t : c->groups[gi].tiles) {
            if (group) group[k] = (int32_t)gi;
            if (b0) b0[k] = t.b0;
            if (b1) b1[k] = t.b1;
            if (nB) nB[k] = t.nB;
            ++k;
        }
    return SNK_OK;
}

int snk_ctx_tile_functions(const snk_ctx* c, int32_t tile, int32_t* fn)
{
    if (!c || !fn) return arg_error(nullptr, "NULL argument");
    int32_t k = 0;
    if (tile >= 0)
        for (const Group& g : c->groups)
            for (const Tile& t : g.tiles)
                if (k++ == tile) {
                    std::copy(t.coll_fn.begin(), t.coll_fn.end(), fn);
                    return SNK_OK;
                }
    return arg_error(nullptr, "tile index out of range");
}

int snk_ctx_block_data(snk_ctx* c, const double* P, float* features, double* block_energy, int32_t* pair_shells)
{
    if (!c || !P) return arg_error(c, "NULL context or density");
    ZeroRows zr(c);
    if (!features && !block_energy && !pair_shells) return SNK_OK;
    const int64_t nbf = c->nbf;
    const int64_t ldk = (int64_t)c->ne_list.size();
    if (pair_shells)
        for (int64_t k = 0; k < ldk; ++k) {
            pair_shells[2 * k] = c->pair_a[c->ne_list[k]];
            pair_shells[2 * k + 1] = c->pair_b[c->ne_list[k]];
        }
    if (!features && !block_energy) return SNK_OK;
    HIPCHECK(c, hipSetDevice(c->device));
    int rc = setup_screening(c);
    if (rc) return rc;
    hipStream_t s = c->stream;
    const double* dP = P;
    if (!(c->opts.flags & SNK_DEVICE_PTRS)) {
        HIPCHECK(c, hipMemcpyAsync(c->d_P, P, (size_t)nbf * nbf * sizeof(double), hipMemcpyHostToDevice, s));
        dP = c->d_P;
    }
    HIPCHECK(c, launch_pair_pnorm(dP, nbf, c->d_ne_list, c->d_pa, c->d_pb, c->d_shell_l, c->d_shell_row,
                                  (int64_t)c->ne_list.size(), c->d_lp, s));
    if (c->mixed) HIPCHECK(c, launch_convert_f32(dP, nbf * nbf, c->d_P32, s));
    if ((rc = link_prepare(c, dP))) return rc;
    for (const Group& g : c->groups) {
        if ((rc = group_F(c, g, dP, false))) return rc;
        if ((rc = group_bounds(c, g))) return rc;
        const int nb = g.b1 - g.b0;
        if (features)
            HIPCHECK(c, launch_block_features(c->d_ne_list, c->d_pa, c->d_pb, (int32_t)ldk, c->d_pfeat, c->d_lp,
                                              c->d_geo + g.b0, c->d_lun, c->nshell, nb,
                                              features + (int64_t)g.b0 * ldk * 16, ldk, s));
        if (block_energy) {
            const int64_t off = (int64_t)g.b0 * kBatch;
            for (int cl = 0; cl < 6; ++cl) {
                const int n = c->ne_class_off[cl + 1] - c->ne_class_off[cl];
                if (n == 0) continue;
                HIPCHECK(c, launch_block_energy(kClassLA[cl], kClassLB[cl], c->d_px + off, c->d_py + off,
                                                c->d_pz + off, c->d_pw + off, c->d_F,
                                                c->mixed ? c->d_F32 : nullptr, g.ncols, c->d_pairs,
                                                c->d_prims, c->d_pfeat, c->d_ne_list + c->ne_class_off[cl], n, nb,
                                                block_energy + (int64_t)g.b0 * ldk + c->ne_class_off[cl], ldk,
                                                c->d_boys, s));
            }
        }
    }
    HIPCHECK(c, hipStreamSynchronize(s));
    return SNK_OK;
}

int snk_collect_block_norms(snk_ctx* c, const double* P, float* feats, float* target, int64_t cap, int64_t* n_out)
{
    if (!c || !P || !feats || !target || !n_out) return arg_error(c, "NULL argument");
    const int64_t n = (int64_t)c->nbatch * (int64_t)c->ne_list.size();
    *n_out = n;
    if (cap < n) return arg_error(c, "capacity smaller than the number of blocks");
    if (n == 0) return SNK_OK;
    HIPCHECK(c, hipSetDevice(c->device));
    double* d_t = nullptr;
    int rc = dalloc(c, &d_t, (size_t)n);
    if (rc) return rc;
    rc = snk_ctx_block_data(c, P, feats, d_t, nullptr);
    if (!rc) {
        hipError_t e = launch_log10(d_t, n, target, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            set_err(c, std::string("block norms: ") + hipGetErrorString(e));
            rc = SNK_E_DEVICE;
        }
    }
    (void)hipFree(d_t);
    return rc;
}

int snk_ctx_debug_learned(snk_ctx* c, const double* P, float* yraw, float* est, int32_t* thr, int64_t* nbatch_out)
{
    if (!c || !P) return arg_error(c, "NULL argument");
    if (!c->mlp) return arg_error(c, "context was not created with SNK_SCREEN_LEARNED");
    if (c->groups.empty()) {
        if (nbatch_out) *nbatch_out = 0;
        return SNK_OK;
    }
    const Group& g = c->groups[0];
    const int64_t nbf = c->nbf;
    const int nb = g.b1 - g.b0;
    // the library keeps estimates by position among the pairs with kept primitive pairs; the
    // outputs are indexed by pair index
    const size_t nne = c->ne_list.size();
    const size_t n = std::max<size_t>(1, (size_t)nb * nne);
    HIPCHECK(c, hipSetDevice(c->device));
    hipStream_t s = c->stream;
    HIPCHECK(c, hipMemcpyAsync(c->d_P, P, (size_t)nbf * nbf * sizeof(double), hipMemcpyHostToDevice, s));
    float* d_y = nullptr;
    int rc = dalloc(c, &d_y, n);
    if (rc) return rc;
    // non-candidate blocks keep NaN
    std::vector<float> nanv(n, std::nanf(""));
    HIPCHECK(c, hipMemcpyAsync(d_y, nanv.data(), n * sizeof(float), hipMemcpyHostToDevice, s));
    HIPCHECK(c, hipMemcpyAsync(c->d_est, nanv.data(), n * sizeof(float), hipMemcpyHostToDevice, s));
    HIPCHECK(c, launch_pair_pnorm(c->d_P, nbf, c->d_ne_list, c->d_pa, c->d_pb, c->d_shell_l, c->d_shell_row,
                                  (int64_t)c->ne_list.size(), c->d_lp, s));
    if (c->mixed) HIPCHECK(c, launch_convert_f32(c->d_P, nbf * nbf, c->d_P32, s));
    if ((rc = link_prepare(c, c->d_P))) return rc;
    GroupStats gs;
    rc = group_until_G(c, g, c->d_P, false, &gs, d_y);
    if (!rc) {
        std::vector<float> hy(n), he(n);
        hipError_t e = hipMemcpyAsync(hy.data(), d_y, n * sizeof(float), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(he.data(), c->d_est, n * sizeof(float), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && thr) e = hipMemcpyAsync(thr, c->d_thr, nb * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            set_err(c, std::string("debug copy: ") + hipGetErrorString(e));
            rc = SNK_E_DEVICE;
        } else {
            const size_t np = (size_t)c->npair_total;
            for (size_t b = 0; b < (size_t)nb; ++b) {
                if (yraw) std::fill(yraw + b * np, yraw + (b + 1) * np, std::nanf(""));
                if (est) std::fill(est + b * np, est + (b + 1) * np, std::nanf(""));
                for (size_t k = 0; k < nne; ++k) {
                    if (yraw) yraw[b * np + c->ne_list[k]] = hy[b * nne + k];
                    if (est) est[b * np + c->ne_list[k]] = he[b * nne + k];
                }
            }
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(d_y);
    if (!rc && nbatch_out) *nbatch_out = nb;
    return rc;
}

int snk_ctx_debug_kept(snk_ctx* c, const double* P, int32_t* out, int64_t cap, int64_t* n_out)
{
    if (!c || !P || !n_out) return arg_error(c, "NULL argument");
    if (c->opts.screen == SNK_SCREEN_NONE) return arg_error(c, "context has no density screen");
    if (c->opts.flags & SNK_DEVICE_PTRS) return arg_error(c, "host-pointer contexts only");
    *n_out = 0;
    if (c->groups.empty()) return SNK_OK;
    const int64_t nbf = c->nbf;
    HIPCHECK(c, hipSetDevice(c->device));
    int rc = setup_screening(c);
    if (rc) return rc;
    hipStream_t s = c->stream;
    HIPCHECK(c, hipMemcpyAsync(c->d_P, P, (size_t)nbf * nbf * sizeof(double), hipMemcpyHostToDevice, s));
    if (c->mixed) HIPCHECK(c, launch_convert_f32(c->d_P, nbf * nbf, c->d_P32, s));
    if (c->mlp)
        HIPCHECK(c, launch_pair_pnorm(c->d_P, nbf, c->d_ne_list, c->d_pa, c->d_pb, c->d_shell_l, c->d_shell_row,
                                      (int64_t)c->ne_list.size(), c->d_lp, s));
    if ((rc = link_prepare(c, c->d_P))) return rc;
    c->d_P_cur = c->d_P;
    GroupStats gs;
    c->kept_capture = true;
    rc = group_until_G(c, c->groups[0], c->d_P, false, &gs);
    c->kept_capture = false;
    if (rc) return rc;
    HIPCHECK(c, hipStreamSynchronize(s));
    const int64_t n = (int64_t)c->kept.size() / 3;
    *n_out = n;
    if (out) {
        if (cap < n) return arg_error(c, "output holds fewer triples than the screen kept");
        std::copy(c->kept.begin(), c->kept.end(), out);
    }
    return SNK_OK;
}

int64_t snk_ctx_npair_index(const snk_ctx* c) { return c ? c->npair_total : 0; }

int snk_debug_mfma_bf16(const float* A, const float* B, float* D, int k32)
{
    if (!A || !B || !D) return arg_error(nullptr, "NULL argument");
    const int na = k32 ? 512 : 256;
    float* d = nullptr;
    if (hipMalloc((void**)&d, (2 * na + 256) * sizeof(float)) != hipSuccess) return SNK_E_NOMEM;
    hipError_t e = hipMemcpy(d, A, na * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d + na, B, na * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = k32 ? launch_mfma_bf16_k32_probe(d, d + na, d + 2 * na, nullptr)
                : launch_mfma_bf16_probe(d, d + na, d + 2 * na, nullptr);
    if (e == hipSuccess) e = hipMemcpy(D, d + 2 * na, 256 * sizeof(float), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) {
        g_last_error = hipGetErrorString(e);
        return SNK_E_DEVICE;
    }
    return SNK_OK;
}

int snk_boys_device(const double* T, int64_t n, int mmax, double* F_out, void* stream)
{
    if (n < 0 || mmax < 0 || mmax > 2 * SNK_MAX_L) return arg_error(nullptr, "bad Boys request");
    if (n == 0) return SNK_OK;
    if (!T || !F_out) return arg_error(nullptr, "NULL pointer");
    static double* d_tab = nullptr;
    static int tab_dev = -1;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SNK_E_DEVICE;
    if (!d_tab || tab_dev != dev) {
        const auto& t = boys_table();
        if (hipMalloc((void**)&d_tab, t.size() * sizeof(double)) != hipSuccess) return SNK_E_NOMEM;
        if (hipMemcpy(d_tab, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
            return SNK_E_DEVICE;
        tab_dev = dev;
    }
    hipError_t e = launch_boys_eval(T, n, mmax, F_out, d_tab, (hipStream_t)stream);
    if (e != hipSuccess) {
        g_last_error = hipGetErrorString(e);
        return SNK_E_DEVICE;
    }
    return SNK_OK;
}

}  // extern "C"

namespace snk {
// error text of a context-free call (snk_last_error(NULL)), for entry points in other files
void set_last_error(const char* msg) { g_last_error = msg ? msg : ""; }

// F_m(T_k), T_k = k kBoysStep (k < kBoysRows), m < cols, by Gauss-Legendre quadrature of the
// defining integral (Eq. boys) in long double; row-major
std::vector<double> boys_table_cols(int cols)
{
    std::vector<long double> gx, gw;
    gauss_legendre(160, gx, gw);
    std::vector<double> tab((size_t)kBoysRows * cols);
    for (int k = 0; k < kBoysRows; ++k) {
        const long double T = (long double)k * kBoysStep;
        for (int m = 0; m < cols; ++m) {
            long double s = 0.0L;
            for (size_t q = 0; q < gx.size(); ++q) {
                const long double y = 0.5L * (gx[q] + 1.0L);
                s += gw[q] * powl(y, 2 * m) * expl(-T * y * y);
            }
            tab[(size_t)k * cols + m] = (double)(0.5L * s);
        }
    }
    return tab;
}
}  // namespace snk
