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

// Every tile of a batch group in one launch: workgroup w belongs to the tile with the largest
// first workgroup wg0 <= w (tile records in workgroup order), and within it to column block
// (w - wg0) % ncb and shell block (w - wg0) / ncb; Phi_t is nB_t x ncols_t at phi_off.
template <typename T>
__global__ __launch_bounds__(256) void collocate_tiles_kernel(const double* __restrict__ px,
                                                              const double* __restrict__ py,
                                                              const double* __restrict__ pz,
                                                              const ShellDev* __restrict__ shells,
                                                              const double* __restrict__ exps,
                                                              const double* __restrict__ coefs,
                                                              const CollTile* __restrict__ tiles, int32_t ntile,
                                                              T* __restrict__ Phi)
{
    const int64_t w = blockIdx.x;
    int lo = 0, hi = ntile - 1;
    while (lo < hi) {   // uniform over the workgroup
        const int mid = (lo + hi + 1) >> 1;
        if (tiles[mid].wg0 <= w) lo = mid;
        else hi = mid - 1;
    }
    const CollTile t = tiles[lo];
    const int64_t lw = w - t.wg0;
    const int cb = (int)(lw % t.ncb), sb = (int)(lw / t.ncb);
    const int64_t col = (int64_t)cb * blockDim.x + threadIdx.x;
    if (col >= t.ncols || sb * kShellsPerBlock >= t.nsh) return;
    const double x = px[t.col0 + col], y = py[t.col0 + col], z = pz[t.col0 + col];
    const int s0 = sb * kShellsPerBlock;
    const int s1 = min(t.nsh, s0 + kShellsPerBlock);
    const int64_t ld = t.ncols;
    for (int si = s0; si < s1; ++si) {
        const ShellDev sh = shells[t.shells[si]];
        const int64_t row = t.rows[si];
        const double dx = x - sh.x, dy = y - sh.y, dz = z - sh.z;
        const double r2 = dx * dx + dy * dy + dz * dz;
        double rad = 0.0;
        for (int k = 0; k < sh.nprim; ++k) rad = fma(coefs[sh.prim_off + k], exp(-exps[sh.prim_off + k] * r2), rad);
        T* out = Phi + t.phi_off + row * ld + col;
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

int64_t collocate_tiles_plan(CollTile* tiles, int32_t ntile)
{
    int64_t nwg = 0;
    for (int i = 0; i < ntile; ++i) {
        tiles[i].ncb = (int32_t)((tiles[i].ncols + 255) / 256);
        tiles[i].wg0 = nwg;
        nwg += (int64_t)tiles[i].ncb * ((tiles[i].nsh + kShellsPerBlock - 1) / kShellsPerBlock);
    }
    return nwg;
}

template <typename T>
static hipError_t launch_collocate_tiles_t(const double* px, const double* py, const double* pz,
                                           const ShellDev* shells, const double* exps, const double* coefs,
                                           const CollTile* tiles, int32_t ntile, int64_t nwg, T* Phi, hipStream_t s)
{
    if (ntile <= 0 || nwg <= 0) return hipSuccess;
    if (nwg > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((collocate_tiles_kernel<T>), dim3((unsigned)nwg), dim3(256), 0, s, px, py, pz, shells, exps,
                       coefs, tiles, ntile, Phi);
    return hipGetLastError();
}

hipError_t launch_collocate_tiles(const double* px, const double* py, const double* pz, const ShellDev* shells,
                                  const double* exps, const double* coefs, const CollTile* tiles, int32_t ntile,
                                  int64_t nwg, double* Phi, hipStream_t s)
{
    return launch_collocate_tiles_t<double>(px, py, pz, shells, exps, coefs, tiles, ntile, nwg, Phi, s);
}

hipError_t launch_collocate_tiles(const double* px, const double* py, const double* pz, const ShellDev* shells,
                                  const double* exps, const double* coefs, const CollTile* tiles, int32_t ntile,
                                  int64_t nwg, float* Phi, hipStream_t s)
{
    return launch_collocate_tiles_t<float>(px, py, pz, shells, exps, coefs, tiles, ntile, nwg, Phi, s);
}

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
