// Internal declarations shared by the host runtime and the HIP kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

namespace snk {

constexpr int kBatch = 256;          // grid points per batch slot (one workgroup, four wave64)
constexpr double kXcRhoMin = 1e-12;  // XC: grid points with a smaller density contribute nothing
constexpr int kMaxL = 2;
constexpr int kMaxNprim = 8;

// Boys table: F_m(T_k), T_k = k * kBoysStep, k = 0..kBoysRows-1, m = 0..kBoysCols-1.
// Taylor expansion about the nearest node with kBoysTerms terms is used for
// T < kBoysTmax; above it the asymptotic form is exact to double precision for m <= 4.
constexpr double kBoysStep = 0.25;
constexpr double kBoysTmax = 50.0;
constexpr int kBoysTerms = 11;                       // j = 0..10
constexpr int kBoysRows = 201;
constexpr int kBoysCols = 2 * kMaxL + kBoysTerms;    // m + j <= 14

// One unique shell pair, oriented so that l_A >= l_B (A = first shell).
struct PairHdr {
    int32_t prim_begin;  // first primitive pair in the PrimPair array
    int32_t nprim;       // surviving primitive pairs
    int32_t fa, fb;      // global index of the first basis function of shells A and B
    double ABx, ABy, ABz;
    double pad;
};

// Centre-independent data of one primitive pair (Obara-Saika, App. A).  The fields an
// s-s pair needs come first so that one 64-byte scalar load covers them.
struct PrimPair {
    double Px, Py, Pz;   // R_p
    double zp;           // zeta_a + zeta_b
    double pref;         // (2 pi / zeta_p) exp(-zeta_a zeta_b |AB|^2 / zeta_p) c_a c_b
    double PAx, PAy, PAz;// R_p - R_A
    double oo2zp;        // 1 / (2 zeta_p)
    double pad;
};

// FP32 copy of a primitive pair for the reduced-precision A.F blocks (same index).
struct PrimPair32 {
    float Px, Py, Pz, zp, pref, PAx, PAy, PAz, oo2zp, pad;
};

struct ShellDev {
    double x, y, z;
    int32_t l, nprim, prim_off, pad;
};

// A.F work of one (l_A, l_B) class is organised in runs.  A run fixes a tile of up
// to kTileA[class] A shells whose F rows and G accumulators stay in registers; it
// lists B tasks, each a B shell with the pairs (a_k, B) of the tile to evaluate.
// Runs and B tasks are int32 records:
//   run:   [b_begin, b_end, arow_0 .. arow_{TA-1}]                 (arow = -1: empty slot)
//   btask: [brow, mask, prim_begin_0, nprim_0, .., prim_begin_{TA-1}, nprim_{TA-1}]
//          (bit k of mask: pair (a_k, B) present; its primitive pairs are
//           prims[prim_begin_k .. prim_begin_k + nprim_k))
// The pair geometry R_A - R_B comes from the shell centres by basis-function row (rowc), the
// same difference the pair table holds.
constexpr int kMaxTile = 8;
constexpr int kTileA[6] = {4, 2, 2, 1, 1, 1};   // ss, ps, pp, ds, dp, dd
// A tiles of the FP32 lists (list 6 + class): FP32 registers are half as wide, so twice the
// tile fits, and each F_B load / G_B update then serves twice the pairs
constexpr int kTileA32[6] = {8, 4, 4, 2, 2, 1};

// class c = ss, ps, pp, ds, dp, dd: (l_A, l_B) and A-tile size, usable in device code
__host__ __device__ constexpr int kClassLA_dev(int c) { return c == 0 ? 0 : (c < 3 ? 1 : 2); }
__host__ __device__ constexpr int kClassLB_dev(int c) { return (c == 0 || c == 1 || c == 3) ? 0 : ((c == 2 || c == 4) ? 1 : 2); }
__host__ __device__ constexpr int kTileA_dev(int c)
{
    return c == 0 ? kTileA[0] : c == 1 ? kTileA[1] : c == 2 ? kTileA[2] : c == 3 ? kTileA[3] : c == 4 ? kTileA[4] : kTileA[5];
}
// tile of screened list k (0-5 FP64 classes, 6-11 FP32 classes)
__host__ __device__ constexpr int kListTile(int k)
{
    return k < 6 ? kTileA_dev(k)
                 : (k == 6 ? kTileA32[0] : k == 7 ? kTileA32[1] : k == 8 ? kTileA32[2] : k == 9 ? kTileA32[3]
                                                              : k == 10 ? kTileA32[4] : kTileA32[5]);
}

struct AfgArgs {
    const double* px;
    const double* py;
    const double* pz;
    const double* pw;
    const double* F;        // [rows][ld]
    const float* F32;       // FP32 F of the mixed-precision build (used instead of F when set)
    double* G;              // [rows][ld]
    int64_t ld;
    const PairHdr* pairs;
    const PrimPair* prims;
    const PrimPair32* prims32;      // FP32 copy of prims
    bool lowp;                      // evaluate in FP32 (reduced-precision blocks)
    const int32_t* runs;            // run records of one class
    const int32_t* btasks;          // B-task records of that class
    const double* rowc;             // [rows][3] centre of the shell of each basis function
    const int32_t* batch_run_off;   // [nbatch+1] per-batch run ranges, or nullptr: all runs for all batches
    int32_t nrun;
    int32_t nbatch;                 // workgroups: batches of the group, or entries of batch_order
    const int32_t* batch_order;     // [nbatch] batch of each workgroup, or nullptr: workgroup w, batch w
    const double* boys_tab;
};

// Density-dependent screening (rigorous bound) of one batch group.
struct ScreenArgs {
    const double* U;            // [nbatch][nshell] block-bound factors
    int32_t nshell;
    int32_t nbatch;
    const int32_t* batch_order; // [nbatch] batch of each workgroup (a permutation), or nullptr: workgroup w, batch w
    const int32_t* shell_l;     // [nshell]
    const int32_t* shell_row;   // [nshell] first row of the shell in F/G
    const PairHdr* pairs;       // unique pairs, index s(s+1)/2 + t for s >= t
    double eps_batch;           // energy budget of the skipped blocks of one batch
    double eps_low;             // estimate budget of the reduced-precision blocks of one batch
    int32_t nlist;              // 6: one list per class; 12: lists 0-5 FP64, lists 6-11 FP32 (same classes)
    int32_t* counts;            // [nbatch][nlist][2]: runs, B tasks
    int64_t* npairs;            // [nbatch][nlist]: shell pairs kept
    double* skipped;            // [nbatch]: bound on the skipped energy
    const int64_t* run_base;    // [nlist][nbatch+1]
    const int64_t* bt_base;     // [nlist][nbatch+1]
    int32_t* runs[12];
    int32_t* btasks[12];
    int32_t* batch_run_off[12]; // [nbatch+1]
    const float* est;           // learned screen: [nbatch][nne] log2 block estimate, or nullptr
    const int32_t* thr;         // learned screen: [nbatch] first kept estimate bin
    const int32_t* thr2;        // learned screen: [nbatch] first FP64 estimate bin (bins thr..thr2-1 are FP32)
    const int32_t* ne_pos;      // [npair_total] position of a pair among the pairs with kept primitive
                                // pairs (the index of est), -1 for a pair without any
    int64_t nne;                // pairs with kept primitive pairs
    int32_t* shell_flag;        // [tiles][nshell]: set to 1 for both shells of every kept block (or nullptr)
    int32_t tile_batches;       // batches per tile (tile of batch b: b / tile_batches)
    // pair selection of Eq. sp_set (link != 0): thresholds and the estimates it takes
    int32_t link;
    double link_eps;            // eps_E = eps_K
    const double* fmax;         // [nbatch][nshell] max_i sqrt(w_i) |F_a,i| over the shell's functions
    const double* phit;         // [nbatch] max_i sqrt(w_i) sum_mu |Phi_mu,i|
    const double* atil;         // [npair_total] global estimate of max |A_ab| of the pair
};

// Relative error allowed for in an FP32-evaluated block of the mixed build: the FP32 set's
// summed estimates times kLowRelErr stay within eps_lowprec_energy.  FP32 rounds at 2^-24;
// the recurrences and the contraction lose up to a few digits more on cancellation.
constexpr double kLowRelErr = 1e-5;
// Split build (SNK_MIXED with basis and density screening): on each tile the functions whose
// largest |Phi| over the tile's points is below kWeakPhi enter F = P Phi and K~ = G Phi^T through
// the FP32 matrix cores.  For such a function |Phi_nu,i| < kWeakPhi, so the FP32 products move
// F_lam,i by at most gamma kWeakPhi sum_{nu weak} |P_lam,nu| and K~_mu,nu by at most
// gamma kWeakPhi sum_i |G_mu,i|; with E_x = -1/2 sum F G this bounds the energy change by
// gamma kWeakPhi sum_t sum_mu (sum_{i in t} |G_mu,i|) (sum_{nu weak on t} |P_mu,nu|).  gamma:
// operands rounded to FP32 (2 u) and FP32 sums of at most 1024 terms (1024 u), u = 2^-24.
constexpr double kWeakPhi = 1e-3;
constexpr double kFp32GemmGamma = (2.0 + 1024.0) / 16777216.0;

// block-energy histograms of the screens: bin = floor(2 log2 e) + kBinOff, clamped to [0, kNBins)
constexpr int kBinOff = 400;
constexpr int kNBins = 512;

// learned screener network 16 -> 64 -> 64 -> 1
constexpr int kMlpIn = 16;
constexpr int kMlpParams = 64 * 16 + 64 + 64 * 64 + 64 + 64 + 1;   // 5313
// samples per call of snk_mlp_loss_grad_noalloc (its fixed scratch array)
constexpr int64_t kMlpNoAllocMaxSamples = 65536;
struct MlpNorm {
    float mean[16];
    float inv_std[16];
};

// Static data of one shell pair used by the learned screener's features (indexed like PairHdr).
struct PairFeat {
    float a[3], b[3];    // centres of shells A and B
    float pc[3];         // centre of the most diffuse primitive pair
    float la, lb;        // angular momenta
    float lzA, lzB;      // log10 of the smallest exponent of A and of B
    float ab;            // |AB|
    float lq;            // log10 sum over kept primitive pairs of |prefactor| (-40 if none)
    float cab;           // 1 for A != B (the block and its transpose), 1/2 for A == B
};

// Static data of one grid batch (valid points only).
struct BatchGeo {
    float lo[3], hi[3];  // bounding box
    float ctr[3];        // centroid
    float hd;            // half diagonal of the box
    float lw;            // log10 of the weight sum (-40 if zero)
    float pad;
};

// Learned estimate pass of one batch group: per batch, every candidate block (pairs the
// rigorous bound does not already skip) gets est = min(bound, 10^(y + margin)) from the
// network (the bound alone when a feature lies outside the training range), stored as
// log2(est) in est[batch][k] (k: the pair's position in the list of pairs with kept primitive
// pairs); the batch's skip threshold bin goes to thr[batch].
struct EstArgs {
    const double* U;            // [nbatch][nshell] bound factors
    const float2* lun;          // [nbatch][nshell] log10 U and log10 of the F norm (clamped at -40)
    int32_t nshell;
    int32_t nbatch;
    const int32_t* batch_order; // [nbatch] batch of each workgroup (a permutation), or nullptr
    const int32_t* shell_l;
    int64_t nne;                // pairs with kept primitive pairs, in class order:
    const int32_t* ne_p;        //   [nne] pair index
    const int2* ne_ab;          //   [nne] shells (A, B)
    const PairFeat* ne_feat;    //   [nne] static features
    const float* ne_lp;         //   [nne] log10 of the Frobenius norm of the P block
    const int32_t* ne_pos;      // [npair_total] position of a pair index in that list, -1 if absent
    const BatchGeo* geo;        // [nbatch] of this group
    double eps_batch;
    const float* params;        // network parameters (FP32; rounded to bf16 on load)
    MlpNorm norm;
    float lo[16], hi[16];       // training range of the raw features
    float margin;               // log10 units added to every prediction
    float* est;                 // [nbatch][nne] log2 of the block estimate
    float* yraw;                // optional [nbatch][nne] raw network output
    int32_t* thr;               // [nbatch] first kept bin of the learned estimate
    double eps_low;             // estimate budget of the reduced-precision blocks of one batch (0: none)
    int32_t* thr2;              // [nbatch] first FP64 bin (bins thr .. thr2-1 go to FP32)
    double* skipped;            // [nbatch] estimated energy of the skipped blocks
};

// launchers (return hipError_t of the launch)
hipError_t launch_mlp_forward(const float* params, const MlpNorm& nrm, const float* x, int64_t n, float* y, bool bf16,
                              hipStream_t s);
int64_t mlp_grad_blocks(int64_t n);
// gradients of the loss (dy == nullptr: asymmetric squared error against target) or of
// sum_s dy[s] y[s] (dy given, target unused) with respect to the parameters; grads[kMlpParams]
// holds the loss (0 in the second form)
hipError_t launch_mlp_grad(const float* params, const MlpNorm& nrm, const float* x, const float* target,
                           const float* dy, int64_t n, float under, float* part, float* grads, hipStream_t s);
// out[k] = log10(in[k]) for in[k] > 1e-40, else -40
hipError_t launch_log10(const double* in, int64_t n, float* out, hipStream_t s);
hipError_t launch_mlp_adam(float* params, float* m, float* v, const float* g, float lr, int t, hipStream_t s);
// U_A (and its log features) of the shells of one angular momentum for the batches of one
// group: one workgroup per batch, lane = point.
struct DiagArgs {
    const double *px, *py, *pz, *pw;   // the group's points
    const int32_t* batch_order;        // [nbatch] batch of each workgroup (a permutation), or nullptr
    const double* F;                   // F of the group (ld columns), or
    const float* F32;                  // its FP32 copy
    int64_t ld;
    const PrimPair32* prims;           // folded same-centre primitive pairs of the diagonal entries
    const int32_t* dsh;                // [n] shell of each diagonal entry
    const int32_t* drow;               // [n] its first basis function
    const int32_t* dpb;                // [n] first primitive-pair record
    const int32_t* dnp;                // [n] number of records
    int32_t n;
    const int32_t* list;               // [ntile][n] per tile, the entries whose shell the tile flags, or nullptr: all
    const int32_t* count;              // [ntile] list lengths
    int32_t tile_batches;
    double* U;                         // [nbatch][nshell]
    float2* lun;                       // [nbatch][nshell] (log10 U, log10 |F_A|), or nullptr
    double* fmax;                      // [nbatch][nshell] max_i sqrt(w_i) |F_A,i|, or nullptr
    int32_t nshell;
    int32_t nbatch;
    const double* tab;                 // Boys table
};
hipError_t launch_diag_bound(int l, const DiagArgs& a, hipStream_t s);
// Per tile and angular momentum l: list[l][t][..] = the diagonal entries k (ascending) with
// flag[t][dsh[l][k]] != 0, count[l][t] their number.
struct DiagLists {
    const int32_t* dsh[3];
    int32_t n[3];
    int32_t* list[3];    // [ntile][n[l]]
    int32_t* count[3];   // [ntile]
};
hipError_t launch_diag_lists(const DiagLists& d, const int32_t* flag, int32_t ntile, int32_t nshell, hipStream_t s);
// phit[b] = max over the points of batch b of sqrt(w_i) sum_mu |Phi_mu,i| for the batches of one
// group: batch b lies in tile t = b / tile_batches, whose Phi_t has rows roff[t]..roff[t+1]-1
// (tiles before the last have tile_batches * 256 columns, the last ncols_last)
// out[b][k] = max over the points i of batch b of sqrt(w_i) |Phi_k,i| for the rows k of the
// batch's tile (tiles and Phi layout as for launch_phisum), row stride ld
hipError_t launch_phimax(const double* Phi, const float* Phi32, const int32_t* roff, int32_t ntile,
                         int32_t tile_batches, int64_t ncols_last, const double* pw, int32_t nbatch, double* out,
                         int64_t ld, hipStream_t s);
// fs[b][A] = max over the functions mu of shell A of Ft[b][mu] (row stride ldf)
hipError_t launch_shellmax(const double* Ft, int64_t ldf, const int32_t* shell_l, const int32_t* shell_row,
                           int32_t nshell, int32_t nbatch, double* fs, hipStream_t s);
hipError_t launch_phisum(const double* Phi, const float* Phi32, const int32_t* roff, int32_t ntile,
                         int32_t tile_batches, int64_t ncols_last, const double* pw, int32_t nbatch, double* phit,
                         hipStream_t s);
hipError_t launch_screen(bool write, const ScreenArgs& a, hipStream_t s);
// Rows of G that the kept blocks of each tile can touch: for tile t, rows[t * nbf + m]
// (m < count[t]) are the functions of the flagged shells in ascending order.
hipError_t launch_tile_rows(const int32_t* shell_flag, int32_t ntile, int32_t nshell, const int32_t* shell_l,
                            const int32_t* shell_row, int32_t nbf, int32_t* rows, int32_t* count, hipStream_t s);
hipError_t launch_screen_est(const EstArgs& a, hipStream_t s);
// lp[k] = log10 ||P_AB|| of the listed pairs plist[k] (pa/pb: shells of each pair index)
hipError_t launch_pair_pnorm(const double* P, int64_t nbf, const int32_t* plist, const int32_t* pa,
                             const int32_t* pb, const int32_t* shell_l, const int32_t* shell_row, int64_t n,
                             float* lp, hipStream_t s);
// training data: features [b][k][16] and exact block energies t[b][k] of the listed pairs
hipError_t launch_block_features(const int32_t* plist, const int32_t* pa, const int32_t* pb, int32_t n,
                                 const PairFeat* pfeat, const float* lp, const BatchGeo* geo, const float2* lun,
                                 int32_t nshell, int32_t nbatch, float* feat, int64_t ldk, hipStream_t s);
hipError_t launch_block_energy(int la, int lb, const double* px, const double* py, const double* pz, const double* pw,
                               const double* F, const float* F32, int64_t ld, const PairHdr* pairs, const PrimPair* prims,
                               const PairFeat* pfeat, const int32_t* plist, int32_t n, int32_t nbatch, double* t,
                               int64_t ldk, const double* tab, hipStream_t s);
// D = A B for 16 x 16 row-major A, B (bf16-exact FP32 values) through one bf16 matrix-core op
hipError_t launch_mfma_bf16_probe(const float* A, const float* B, float* D, hipStream_t s);
// D = A B for 16 x 32 A and 32 x 16 B (row-major, bf16-exact) through one 16x16x32 bf16 op
hipError_t launch_mfma_bf16_k32_probe(const float* A, const float* B, float* D, hipStream_t s);
hipError_t launch_screen_scan(const int32_t* counts, int32_t nbatch, int32_t nlist, int64_t* run_base,
                              int64_t* bt_base, hipStream_t s);
hipError_t launch_afg(int la, int lb, const AfgArgs& a, hipStream_t s);
// One tile of a grouped collocation launch (Eq. collocation): columns col0 .. col0 + ncols - 1
// of the group's points, shells[k] written to rows rows[k].. of Phi_t (nB x ncols at phi_off)
struct CollTile {
    int64_t col0, ncols, phi_off;
    const int32_t* shells;
    const int32_t* rows;
    int32_t nsh, ncb;     // shells; column blocks (set by collocate_tiles_plan)
    int64_t wg0;          // first workgroup (set by collocate_tiles_plan)
};
// fills ncb and wg0 of every tile in order; returns the workgroups of the launch
int64_t collocate_tiles_plan(CollTile* tiles, int32_t ntile);
hipError_t launch_collocate_tiles(const double* px, const double* py, const double* pz, const ShellDev* shells,
                                  const double* exps, const double* coefs, const CollTile* tiles, int32_t ntile,
                                  int64_t nwg, double* Phi, hipStream_t s);
hipError_t launch_collocate_tiles(const double* px, const double* py, const double* pz, const ShellDev* shells,
                                  const double* exps, const double* coefs, const CollTile* tiles, int32_t ntile,
                                  int64_t nwg, float* Phi, hipStream_t s);
hipError_t launch_collocate(const double* px, const double* py, const double* pz, int64_t ncols,
                            const ShellDev* shells, const double* exps, const double* coefs,
                            const int32_t* shell_list, const int32_t* shell_row, int32_t nsh,
                            double* Phi, int64_t ld, hipStream_t s);
hipError_t launch_collocate(const double* px, const double* py, const double* pz, int64_t ncols,
                            const ShellDev* shells, const double* exps, const double* coefs,
                            const int32_t* shell_list, const int32_t* shell_row, int32_t nsh,
                            float* Phi, int64_t ld, hipStream_t s);
// Grouped products (k_ggemm.hip).  One problem: for i < M, j < N and chunk z of k,
//   C[z * cstride + crow(i) * ldc + j] = sum_k A[arow(i) * lda + acol(k)] B(k, j)
// with arow, acol, crow the identity where null, B(k, j) = B[k * ldb + j] (row-major) or
// B[j * ldb + k] (bt); the k range [0, K) is cut into ksplit chunks of kchunk.  The host
// fills the operands, sizes and ksplit; ggemm_plan sets kchunk, tm, tn and vec, and wg0 is the
// problem's first workgroup in the launch (sum of ggemm_workgroups of the problems before it).
struct GemmProb {
    const void* A;
    const int32_t* arow;
    const int32_t* acol;
    int64_t lda;
    const void* B;
    const int32_t* bmap;   // rows of B read through this map: B(k, j) = B[bmap(k) ldb + j] (bt: B[bmap(j) ldb + k])
    int64_t ldb;
    void* C;
    const int32_t* crow;
    int64_t ldc;
    int64_t cstride;
    int64_t wg0;
    int32_t M, N, K, ksplit, kchunk, tm, tn;
    int32_t vec;   // bit 0: A rows 16-byte aligned, bit 1: B rows (set by ggemm_plan); bit 2: C += product;
                   // bits 3, 4: A2, B2 rows aligned (set by ggemm_plan)
    // split products only (launch_gsplit): + A2 B2 over K2 more k, FP32 operands, A2 row-major
    // (rows arow(i), stride lda2), B2 row-major K2 x N (stride ldb2)
    const void* A2;
    const void* B2;
    int64_t lda2, ldb2;
    int32_t K2, pad2;
};
constexpr int32_t kGemmAccumulate = 4;
constexpr int kFp32MaxK = 1024;   // longest FP32 sum of a product element
// One tile of a grouped reduction: T[r][ccol(n)] += sum_z part[poff + z M N + rinv(r) N + n]
// for every row r with rinv(r) >= 0 (rinv null: r < M), in list order.
struct RedTile {
    int64_t poff;
    int32_t M, N, ksplit, pad;
    const int32_t* rinv;
    const int32_t* ccol;
};
// Output tiles of the grouped products (rows x columns per workgroup)
constexpr int kTile64 = 64;         // 64 x 64
constexpr int kTile128 = 128;       // 128 x 128
constexpr int kTile64x128 = 192;    // 64 x 128
constexpr int kTile128x256 = 384;   // 128 x 256 (workgroups of 512 threads)
inline int tile_rows(int tile) { return tile == kTile128 || tile == kTile128x256 ? 128 : 64; }
inline int tile_cols(int tile) { return tile == kTile64 ? 64 : (tile == kTile128x256 ? 256 : 128); }
// Output tile for a launch of these problems (M, N and K filled in): 128 x 128 unless a
// smaller tile saves most of the padded work; g_force_tile (a test hook, 0 = off) overrides it
int ggemm_tile(const GemmProb* probs, int nprob);
extern int g_force_tile;
// asize, bsize: bytes per element of A and B
void ggemm_plan(GemmProb& p, int tile, int asize, int bsize);
int64_t ggemm_workgroups(const GemmProb& p);
// probs: device array of nprob problems planned for the tile size, nwg workgroups in all;
// FP64 matrix cores
hipError_t launch_ggemm_f64(const GemmProb* probs, int nprob, int64_t nwg, int tile, bool bt, hipStream_t s);
// FP32 matrix-core forms: operands rounded to FP32 and FP32 sums over each workgroup's k chunk,
// which the caller keeps at most kFp32MaxK long (ksplit), the chunks then added in FP64 by the
// reduction; f32: FP32 A, B, C; f32_dA: FP64 A, FP32 B, FP64 C
hipError_t launch_ggemm_f32(const GemmProb* probs, int nprob, int64_t nwg, int tile, bool bt, hipStream_t s);
hipError_t launch_ggemm_f32_dA(const GemmProb* probs, int nprob, int64_t nwg, int tile, bool bt, hipStream_t s);
// Split products (B row-major, one chunk, overwrite C): FP64 A B over K plus FP32 A2 B2 over
// K2 <= kFp32MaxK, written once in FP64
hipError_t launch_gsplit(const GemmProb* probs, int nprob, int64_t nwg, int tile, hipStream_t s);
// FP32 matrix cores on FP64 operands rounded as they are staged, FP64 C
hipError_t launch_ggemm_f32_dd(const GemmProb* probs, int nprob, int64_t nwg, int tile, bool bt, hipStream_t s);
// One tile of a grouped gather: out[out_off + i ld + k] = src[src_off + rows(i) src_ld + cols(k)]
// for i < M, k < N (rows, cols null: identity), converted to the output type
struct GatherTile {
    int64_t out_off;
    int64_t src_off;
    int64_t src_ld;
    const int32_t* rows;
    const int32_t* cols;
    int32_t M, N, ld, pad;
};
hipError_t launch_gather_tiles(const double* src, const GatherTile* tiles, int ntile, int32_t max_rows, double* out,
                               hipStream_t s);
hipError_t launch_gather_tiles(const float* src, const GatherTile* tiles, int ntile, int32_t max_rows, float* out,
                               hipStream_t s);
hipError_t launch_gather_tiles(const double* src, const GatherTile* tiles, int ntile, int32_t max_rows, float* out,
                               hipStream_t s);
// Per tile t (rows roff[t] .. roff[t+1] of a group's Phi, row maxima mx): perm lists the rows
// with mx >= tau in order, then the others in order (same offsets as the rows); cperm[k] =
// fn[roff[t] + perm[k]] (the function of each permuted row); nstrong[t] = the rows with
// mx >= tau, raised so that at most kFp32MaxK rows follow (the weak rows, k >= nstrong[t])
hipError_t launch_partition(const double* mx, const int32_t* fn, const int32_t* roff, int ntile, double tau,
                            int32_t* perm, int32_t* cperm, int32_t* nstrong, hipStream_t s);
// Bound of the energy error of the FP32 products of a group (the weak rows k >= nstrong[t] of
// each tile): acc[0] += sum over tiles t and the tile's G rows r = rows[t * nbf + 0 .. counts[t])
// of (sum_{i < ncols_t} |G[r][col0_t + i]|) (sum_{k >= nstrong[t]} |P[r][cperm[roff_t + k]]|);
// partials: kBoundChunks doubles per tile of scratch
struct BoundTile {
    int64_t col0;
    int32_t ncols, roff, nB, nstrong;
};
hipError_t launch_lowprec_bound(const double* G, int64_t ld, const double* P, int64_t nbf, const BoundTile* tiles,
                                int ntile, const int32_t* rows, const int32_t* counts, const int32_t* cperm,
                                double* partials, double* acc, hipStream_t s);
constexpr int kBoundChunksPerTile = 32;
// T (nrow rows of stride ldt) += the tiles' chunk sums, one workgroup per row, tiles in order
hipError_t launch_group_reduce(const double* part, const RedTile* tiles, int ntile, double* T, int64_t ldt,
                               int64_t nrow, hipStream_t s);
// rinv[t][r] = position of r in tile t's row list (lists[roff[t] .. roff[t+1]) when roff is
// given, else lists[t * stride .. t * stride + counts[t])), -1 for rows not listed
hipError_t launch_rinv(const int32_t* lists, int64_t stride, const int32_t* roff, const int32_t* counts, int ntile,
                       int64_t nbf, int64_t max_count, int32_t* rinv, hipStream_t s);
hipError_t launch_convert_f32(const double* in, int64_t n, float* out, hipStream_t s);
// Density-fitted Coulomb matrix (Sec. II.B): records and launchers of the J-engine kernels.
constexpr int kDfjBoysCols = 6 + kBoysTerms;   // F_m up to m = 2 + 2 + 2 with the Taylor terms
constexpr int kDfjHerm = 35;                   // Hermite components up to l_a + l_b = 4
constexpr int kDfjAuxHerm = 10;                // ... up to l_c = 2
constexpr int kDfjCart = 36;                   // Cartesian pair components up to (d, d)
// one orbital primitive pair (shells oriented l_A >= l_B)
struct DfjPrim {
    double Px, Py, Pz;     // product centre
    double za, zb;         // exponents
    double ABx, ABy, ABz;  // R_A - R_B
    double cc;             // c_a c_b, doubled for A != B (both orders of the pair in the density sum)
    double cc1;            // c_a c_b
    int32_t fa, fb;        // first basis functions of A and B
};
// one orbital shell pair: its primitive pairs are records pbeg .. pbeg + np - 1
struct DfjShellPair {
    int32_t fa, fb, la, lb, pbeg, np;
};
// one auxiliary shell (one primitive)
struct DfjAux {
    double x, y, z, z_exp, coef;
    int32_t l, f0;
};
hipError_t launch_dfj_hdens(int cls, const DfjPrim* pp, int32_t n, const double* P, int64_t nbf, double* Dh,
                            hipStream_t s);
hipError_t launch_dfj_vaux(int LP, int LC, const DfjPrim* pp, const double* Dh, int32_t pbeg, int32_t pend,
                           int32_t chunk, int32_t slot0, const DfjAux* aux, int32_t abeg, int32_t aend, int32_t nslot,
                           const double* tab, double* part, hipStream_t s);
hipError_t launch_dfj_vfinish(const DfjAux* aux, int32_t naux, const double* part, int32_t nslot, double* v,
                              hipStream_t s);
hipError_t launch_dfj_auxdens(const DfjAux* aux, int32_t naux, const double* d, double* Dc, hipStream_t s);
// workgroup rows over the auxiliary shells of a J digestion launch of n primitive pairs
int dfj_jpair_chunks(int32_t n, int32_t naux);
// Eq. J_df per primitive pair of one class; Jh: workspace of dfj_jpair_chunks(n, naux) * n *
// nherm(l_A + l_B) doubles
hipError_t launch_dfj_jpair(int cls, const DfjPrim* pp, int32_t n, const DfjAux* aux, int32_t naux, const double* Dc,
                            const int32_t* lbeg, const double* tab, double* Jh, double* Jpp, hipStream_t s);
hipError_t launch_dfj_jcollect(const DfjShellPair* sp, int32_t nsp, const double* Jpp, double* J, int64_t nbf,
                               hipStream_t s);
hipError_t launch_dfj_metric(const DfjAux* aux, int32_t naux, const double* tab, double* V, int64_t n, hipStream_t s);
// in place: the lower triangle of A becomes L (A = L L^T); status set to 1 when A is not
// positive definite
hipError_t launch_dfj_cholesky(double* A, int64_t n, int32_t* status, hipStream_t s);
// in place: L becomes L^-1 (lower), W = L^-T (upper); n workgroups, set-up only
hipError_t launch_dfj_invert(double* L, int64_t n, double* W, hipStream_t s);
// d = W (Linv v) with Linv = L^-1, W = L^-T: two triangular products (y holds Linv v)
hipError_t launch_dfj_solve(const double* Linv, const double* W, int64_t n, const double* v, double* y, double* d,
                            hipStream_t s);
hipError_t launch_dfj_dot(const double* a, const double* b, int64_t n, double* out, hipStream_t s);

// Boys table F_m(T_k), k < kBoysRows, m < cols (host, long-double quadrature)
std::vector<double> boys_table_cols(int cols);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s);
// out[k] = |in[k]|
hipError_t launch_abs(const double* in, int64_t n, double* out, hipStream_t s);
hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s);
hipError_t launch_fill(int32_t* p, int64_t n, int32_t v, hipStream_t s);
// p[r * ld + c] = v for r < rows, c < cols
hipError_t launch_fill2d(double* p, int64_t rows, int64_t cols, int64_t ld, double v, hipStream_t s);
hipError_t launch_fill2d(float* p, int64_t rows, int64_t cols, int64_t ld, float v, hipStream_t s);
hipError_t launch_mfma_probe(double* out_dev, hipStream_t s);
// K = (Kt + Kt^T)/2 and ex = -1/2 tr(P K) (two-stage deterministic reduction, partial buffer of nblk doubles)
hipError_t launch_finish(const double* Kt, const double* P, double* K, int64_t nbf, double* partial, int nblk,
                         double* ex, hipStream_t s);
// XC potential (Sec. II.C): Phi (nbf rows, ld = ncols); per point rho, grad rho, the
// functional and G = 2 Z from F and the basis values recomputed from the shells; per point
// w eps and w rho in
// epart[0..ncols) and epart[ncols..2 ncols); fixed-order sums of those into out[0..1]
// (partial: 512 doubles), added to out when accumulate.
hipError_t launch_xc_collocate(const double* px, const double* py, const double* pz, int64_t ncols,
                               const ShellDev* shells, const double* exps, const double* coefs,
                               const int32_t* shell_row, int32_t nsh, double* Phi, hipStream_t s);
// One tile of an XC launch: its F and G rows start at phi_off (row stride ncols), its shells
// are shell_cat[sh_off .. sh_off + nsh) in row order.  Tile k covers columns
// [k * tile_batches * kBatch, ...) of the launch.
struct XcTile {
    int64_t phi_off;
    int32_t ncols, sh_off, nsh, pad;
};
hipError_t launch_xc_point(const double* px, const double* py, const double* pz, const double* pw, int64_t ncols,
                           const ShellDev* shells, const double* exps, const double* coefs, const XcTile* tiles,
                           const int32_t* shell_cat, int32_t tile_batches, const double* F, int fn, double* G,
                           double* epart, hipStream_t s);
hipError_t launch_xc_sum(const double* epart, int64_t n, double* partial, double* out, bool accumulate, hipStream_t s);
hipError_t launch_boys_eval(const double* T, int64_t n, int mmax, double* F, const double* tab, hipStream_t s);
// every tile t < ntile of a group in one launch: rows rows[t * stride + m], m < count[t] (device),
// of p over columns cols[2t] .. cols[2t] + cols[2t + 1] - 1 set to v; max_rows >= every count
hipError_t launch_fill_rows_tiles(double* p, int64_t ld, const int32_t* rows, int64_t stride, const int32_t* count,
                                  const int64_t* cols, int32_t ntile, int32_t max_rows, double v, hipStream_t s);
// p[rows[m] * ld + c] = v for m < M, c < ncols
hipError_t launch_fill_rows(double* p, int64_t ld, const int32_t* rows, int64_t M, int64_t ncols, double v,
                            hipStream_t s);
// Row maxima of a group's Phi buffer: nfull rows of ncols_full columns, then rows nfull..nrow-1
// of ncols_last columns; mx[r] = max_c |Phi_r,c|
hipError_t launch_row_absmax(const double* Phi, int64_t nfull, int64_t ncols_full, int64_t nrow, int64_t ncols_last,
                             double* mx, hipStream_t s);
hipError_t launch_row_absmax(const float* Phi, int64_t nfull, int64_t ncols_full, int64_t nrow, int64_t ncols_last,
                             double* mx, hipStream_t s);
// flag[t * nshell + shell_of[lam]] = 1 where sum_{k in roff[t]..roff[t+1]-1} |P[lam][fn[k]]| mx[k] >= eps
// (a bound on |F_lam| over tile t), for every function lam and tile t < ntile
hipError_t launch_ftilde_flag(const double* P, int64_t nbf, const int32_t* fn, const int32_t* roff, int32_t ntile,
                              const double* mx, double eps, const int32_t* shell_of, int32_t nshell, int32_t* flag,
                              hipStream_t s, const int32_t* cand = nullptr, int64_t cand_stride = 0,
                              const int32_t* ncand = nullptr);
// pmax[a][b] = max |P| over the block of rows a and columns b (blocks of consecutive functions
// blk_fn0[a] .. blk_fn0[a+1]-1; the basis functions of one centre)
hipError_t launch_pblock_max(const double* P, int64_t nbf, const int32_t* blk_fn0, int32_t nblk, double* pmax,
                             hipStream_t s);
// per tile, the functions whose F-row bound can reach eps by the block bound (cand[t][0 ..
// ncand[t]-1], cand_stride >= nbf)
hipError_t launch_ftilde_cand(const int32_t* fn, const int32_t* roff, const double* mx, int32_t ntile,
                              const int32_t* fn_blk, const int32_t* blk_fn0, int32_t nblk, const double* pmax,
                              double eps, int64_t nbf, int32_t* cand, int64_t cand_stride, int32_t* ncand,
                              hipStream_t s);

}  // namespace snk
