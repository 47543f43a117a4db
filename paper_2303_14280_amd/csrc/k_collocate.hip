// Collocation Phi_{mu i} = phi_mu(r_i) (Eq. collocation) for the basis functions of
// one batch group, written function-major: Phi[row(mu)][column(i)] with columns
// padded to whole 256-point batches.  One lane per grid point, a strip of shells
// per workgroup; contracted radial part sum_k c_k exp(-zeta_k r^2) once per shell,
// Cartesian monomials per component (lexicographic order, unit-normalised).  Values are
// formed in FP64 and stored as FP64 or, for the mixed-precision build, FP32.
#include "snk_internal.h"

namespace snk {
namespace {

constexpr int kShellsPerBlock = 8;

template <typename T>
__global__ __launch_bounds__(256) void collocate_kernel(const double* __restrict__ px, const double* __restrict__ py,
                                                        const double* __restrict__ pz, int64_t ncols,
                                                        const ShellDev* __restrict__ shells,
                                                        const double* __restrict__ exps,
                                                        const double* __restrict__ coefs,
                                                        const int32_t* __restrict__ shell_list,
                                                        const int32_t* __restrict__ shell_row, int32_t nsh,
                                                        T* __restrict__ Phi, int64_t ld)
{
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= ncols) return;
    const double x = px[col], y = py[col], z = pz[col];
    const int s0 = blockIdx.y * kShellsPerBlock;
    const int s1 = min(nsh, s0 + kShellsPerBlock);
    for (int si = s0; si < s1; ++si) {
        const ShellDev sh = shells[shell_list[si]];
        const int64_t row = shell_row[si];
        const double dx = x - sh.x, dy = y - sh.y, dz = z - sh.z;
        const double r2 = dx * dx + dy * dy + dz * dz;
        double rad = 0.0;
        for (int k = 0; k < sh.nprim; ++k) rad = fma(coefs[sh.prim_off + k], exp(-exps[sh.prim_off + k] * r2), rad);
        T* out = Phi + row * ld + col;
        if (sh.l == 0) {
            out[0] = (T)rad;
        } else if (sh.l == 1) {
            out[0] = (T)(dx * rad);
            out[ld] = (T)(dy * rad);
            out[2 * ld] = (T)(dz * rad);
        } else {
            const double s3 = 1.7320508075688772 * rad;
            out[0] = (T)(dx * dx * rad);
            out[ld] = (T)(dx * dy * s3);
            out[2 * ld] = (T)(dx * dz * s3);
            out[3 * ld] = (T)(dy * dy * rad);
            out[4 * ld] = (T)(dy * dz * s3);
            out[5 * ld] = (T)(dz * dz * rad);
        }
    }
}

}  // namespace

template <typename T>
static hipError_t launch_collocate_t(const double* px, const double* py, const double* pz, int64_t ncols,
                                     const ShellDev* shells, const double* exps, const double* coefs,
                                     const int32_t* shell_list, const int32_t* shell_row, int32_t nsh, T* Phi,
                                     int64_t ld, hipStream_t s)
{
    if (ncols <= 0 || nsh <= 0) return hipSuccess;
    dim3 grid((unsigned)((ncols + 255) / 256), (unsigned)((nsh + kShellsPerBlock - 1) / kShellsPerBlock)), block(256);
    hipLaunchKernelGGL((collocate_kernel<T>), grid, block, 0, s, px, py, pz, ncols, shells, exps, coefs, shell_list,
                       shell_row, nsh, Phi, ld);
    return hipGetLastError();
}

hipError_t launch_collocate(const double* px, const double* py, const double* pz, int64_t ncols,
                            const ShellDev* shells, const double* exps, const double* coefs,
                            const int32_t* shell_list, const int32_t* shell_row, int32_t nsh, double* Phi,
                            int64_t ld, hipStream_t s)
{
    return launch_collocate_t<double>(px, py, pz, ncols, shells, exps, coefs, shell_list, shell_row, nsh, Phi, ld, s);
}

hipError_t launch_collocate(const double* px, const double* py, const double* pz, int64_t ncols,
                            const ShellDev* shells, const double* exps, const double* coefs,
                            const int32_t* shell_list, const int32_t* shell_row, int32_t nsh, float* Phi,
                            int64_t ld, hipStream_t s)
{
    return launch_collocate_t<float>(px, py, pz, ncols, shells, exps, coefs, shell_list, shell_row, nsh, Phi, ld, s);
}

}  // namespace snk
