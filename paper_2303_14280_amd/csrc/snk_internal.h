// Internal declarations shared by the host runtime and the HIP kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace snk {

constexpr int kBatch = 256;          // grid points per batch slot (one workgroup, four wave64)
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

struct ShellDev {
    double x, y, z;
    int32_t l, nprim, prim_off, pad;
};

// A.F work of one (l_A, l_B) class is organised in runs.  A run fixes a tile of up
// to kTileA[class] A shells whose F rows and G accumulators stay in registers; it
// lists B tasks, each a B shell with the pairs (a_k, B) of the tile to evaluate.
// Runs and B tasks are int32 records, with the pair geometry beside them:
//   run:   [b_begin, b_end, arow_0 .. arow_{TA-1}]                 (arow = -1: empty slot)
//   btask: [brow, mask, prim_begin_0, nprim_0, .., prim_begin_{TA-1}, nprim_{TA-1}]
//          (bit k of mask: pair (a_k, B) present; its primitive pairs are
//           prims[prim_begin_k .. prim_begin_k + nprim_k))
//   btask_ab: [btask][k][3] doubles, R_A - R_B of pair k
constexpr int kMaxTile = 8;
constexpr int kTileA[6] = {4, 2, 2, 1, 1, 1};   // ss, ps, pp, ds, dp, dd

struct AfgArgs {
    const double* px;
    const double* py;
    const double* pz;
    const double* pw;
    const double* F;        // [rows][ld]
    double* G;              // [rows][ld]
    int64_t ld;
    const PairHdr* pairs;
    const PrimPair* prims;
    const int32_t* runs;            // run records of one class
    const int32_t* btasks;          // B-task records of that class
    const double* btask_ab;         // R_A - R_B per B task and tile slot
    const int32_t* batch_run_off;   // [nbatch+1] per-batch run ranges, or nullptr: all runs for all batches
    int32_t nrun;
    int32_t nbatch;
    const double* boys_tab;
};

// launchers (return hipError_t of the launch)
hipError_t launch_afg(int la, int lb, const AfgArgs& a, hipStream_t s);
hipError_t launch_collocate(const double* px, const double* py, const double* pz, int64_t ncols,
                            const ShellDev* shells, const double* exps, const double* coefs,
                            const int32_t* shell_list, const int32_t* shell_row, int32_t nsh,
                            double* Phi, int64_t ld, hipStream_t s);
// C[M x N] = A[M x K] * op(B); A row-major (lda); B row-major K x N (ldb) or, with bt, N x K.
// With nsplit > 1 the K range is cut into nsplit chunks and chunk z writes C + z * split_stride.
hipError_t launch_gemm_f64(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* B,
                           int64_t ldb, bool bt, double* C, int64_t ldc, int nsplit, int64_t split_stride,
                           hipStream_t s);
// Kt[rows[m] * nbf + cols[n]] += sum_z part[z * stride + m * N + n]
hipError_t launch_reduce_scatter(const double* part, int nsplit, int64_t stride, int64_t M, int64_t N,
                                 const int32_t* rows, const int32_t* cols, double* Kt, int64_t nbf, hipStream_t s);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s);
hipError_t launch_mfma_probe(double* out_dev, hipStream_t s);
// K = (Kt + Kt^T)/2 and ex = -1/2 tr(P K) (two-stage deterministic reduction, partial buffer of nblk doubles)
hipError_t launch_finish(const double* Kt, const double* P, double* K, int64_t nbf, double* partial, int nblk,
                         double* ex, hipStream_t s);
hipError_t launch_boys_eval(const double* T, int64_t n, int mmax, double* F, const double* tab, hipStream_t s);
// gather P_g[m][n] = P[rows[m]][cols[n]] (NULL rows/cols: identity)
hipError_t launch_gather(const double* P, int64_t nbf, const int32_t* rows, int64_t M, const int32_t* cols,
                         int64_t N, double* out, hipStream_t s);

}  // namespace snk
