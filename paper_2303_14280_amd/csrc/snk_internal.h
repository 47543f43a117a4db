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

// Centre-independent data of one primitive pair (Obara-Saika, App. A).
struct PrimPair {
    double zp;           // zeta_a + zeta_b
    double oo2zp;        // 1 / (2 zeta_p)
    double Px, Py, Pz;   // R_p
    double PAx, PAy, PAz;// R_p - R_A
    double pref;         // (2 pi / zeta_p) exp(-zeta_a zeta_b |AB|^2 / zeta_p) c_a c_b
    double pad;
};

// A unit of A.F work: one shell pair, with the rows of its two shells in F/G.
struct PairTask {
    int32_t pair;
    int32_t arow;        // row of the first function of shell A in the group's F and G
    int32_t brow;
    int32_t pad;
};

struct ShellDev {
    double x, y, z;
    int32_t l, nprim, prim_off, pad;
};

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
    const PairTask* tasks;  // tasks of one class
    const int32_t* batch_task_off;  // [nbatch+1] per-batch task ranges, or nullptr: all tasks for all batches
    int32_t ntask;
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
