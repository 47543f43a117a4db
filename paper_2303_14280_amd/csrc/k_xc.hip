// Exchange-correlation potential matrix on the grid (Sec. II.C): the kernels between the
// F GEMM (Eq. fmat) and the Z Phi^T GEMM (Eq. vxc_num).
//   * xc_collocate_kernel: Phi (function-major like the sn-K collocation) for the two GEMMs;
//   * xc_point_kernel: one lane per grid point; rho and grad rho from F and the basis values
//     (Eq. den_grid), recomputed in registers, the functional and its partial derivatives
//     E^rho, E^gamma (Eq. exc_grid) in closed form, and the product rows G = 2 Z (Eq. zmat),
//     so that V = (G Phi^T + Phi G^T) / 2 goes through the same symmetrising finish as sn-K;
//   * xc_sum_kernel: fixed-order two-stage sums of w_i eps_i (E_xc) and w_i rho_i (N_el).
// All arithmetic is FP64.  Points with rho below kXcRhoMin contribute nothing.
#include "snk.h"
#include "snk_internal.h"

namespace snk {
namespace {

constexpr int kXcShellsPerBlock = 8;

// ---- functionals: energy per volume e(rho, sigma) and its partial derivatives -------------

constexpr double kPi = 3.14159265358979323846;
constexpr double kCx = 0.73855876638202240588;           // (3/4)(3/pi)^(1/3)
constexpr double kPwA = 0.031091, kPwA1 = 0.21370;
constexpr double kPwB1 = 7.5957, kPwB2 = 3.5876, kPwB3 = 1.6382, kPwB4 = 0.49294;
constexpr double kKappa = 0.804;
constexpr double kBeta = 0.06672455060314922;
constexpr double kMu = kBeta * kPi * kPi / 3.0;
constexpr double kGam = 0.031090690869654895;             // (1 - ln 2) / pi^2

struct XcVal {
    double e, vr, vs;
};

__device__ __forceinline__ void slater(double rho, double& e, double& vr)
{
    const double r13 = cbrt(rho);
    e = -kCx * rho * r13;
    vr = -(4.0 / 3.0) * kCx * r13;
}

// Perdew-Wang 1992 correlation energy per particle (zeta = 0) and its rs derivative
__device__ __forceinline__ void pw92(double rs, double& ec, double& dec)
{
    const double srs = sqrt(rs);
    const double q0 = -2.0 * kPwA * (1.0 + kPwA1 * rs);
    const double q1 = 2.0 * kPwA * (kPwB1 * srs + kPwB2 * rs + kPwB3 * rs * srs + kPwB4 * rs * rs);
    const double dq1 = kPwA * (kPwB1 / srs + 2.0 * kPwB2 + 3.0 * kPwB3 * srs + 4.0 * kPwB4 * rs);
    const double lg = log1p(1.0 / q1);
    ec = q0 * lg;
    dec = -2.0 * kPwA * kPwA1 * lg - q0 * dq1 / (q1 * (q1 + 1.0));
}

__device__ XcVal functional_eval(int fn, double rho, double sigma)
{
    XcVal v{0.0, 0.0, 0.0};
    double ex, vx;
    slater(rho, ex, vx);
    if (fn == SNK_XC_SLATER) {
        v.e = ex;
        v.vr = vx;
        return v;
    }
    const double rs = cbrt(3.0 / (4.0 * kPi * rho));
    double ec, dec;
    pw92(rs, ec, dec);
    const double dec_drho = -dec * rs / (3.0 * rho);
    if (fn == SNK_XC_LDA) {
        v.e = ex + rho * ec;
        v.vr = vx + ec + rho * dec_drho;
        return v;
    }
    // PBE exchange: e_x = e_x^LDA F(s^2)
    const double kf = cbrt(3.0 * kPi * kPi * rho);
    const double ds2_dsig = 1.0 / (4.0 * kf * kf * rho * rho);
    const double s2 = sigma * ds2_dsig;
    const double den = 1.0 + kMu * s2 / kKappa;
    const double Fx = 1.0 + kKappa - kKappa / den;
    const double dFx = kMu / (den * den);
    const double ex_e = ex * Fx;
    const double ex_r = vx * Fx + ex * dFx * (-(8.0 / 3.0) * s2 / rho);
    const double ex_s = ex * dFx * ds2_dsig;
    // PBE correlation: e_c = rho (eps_c + H(eps_c, t^2))
    const double ks2 = 4.0 * kf / kPi;
    const double dt2_dsig = 1.0 / (4.0 * ks2 * rho * rho);
    const double t2 = sigma * dt2_dsig;
    const double B = kBeta / kGam;
    const double E = exp(-ec / kGam);
    const double A = B / expm1(-ec / kGam);
    const double dA_dec = A * A * E / kBeta;
    const double y = A * t2;
    const double D = 1.0 + y + y * y;
    const double Rr = (1.0 + y) / D;
    const double dR_dy = -y * (2.0 + y) / (D * D);
    const double X = 1.0 + B * t2 * Rr;
    const double H = kGam * log(X);
    const double dH_dt2 = kGam * B * (Rr + t2 * A * dR_dy) / X;
    const double dH_dA = kGam * B * t2 * t2 * dR_dy / X;
    const double dH_drho = dH_dA * dA_dec * dec_drho + dH_dt2 * (-(7.0 / 3.0) * t2 / rho);
    v.e = ex_e + rho * (ec + H);
    v.vr = ex_r + ec + H + rho * (dec_drho + dH_drho);
    v.vs = ex_s + rho * dH_dt2 * dt2_dsig;
    return v;
}

// Values (and for GGA gradients) of the Cartesian components of one shell at displacement d,
// in lexicographic order; nc = the component normalisations.
template <bool GGA>
__device__ __forceinline__ int shell_values(const ShellDev& sh, const double* __restrict__ exps,
                                            const double* __restrict__ coefs, double dx, double dy, double dz,
                                            double (&v)[6], double (&gx)[6], double (&gy)[6], double (&gz)[6])
{
    const double r2 = dx * dx + dy * dy + dz * dz;
    double R = 0.0, dR = 0.0;
    for (int k = 0; k < sh.nprim; ++k) {
        const double g = coefs[sh.prim_off + k] * exp(-exps[sh.prim_off + k] * r2);
        R += g;
        dR = fma(-2.0 * exps[sh.prim_off + k], g, dR);
    }
    // monomials m and their derivatives, component by component
    auto put = [&](int i, double nc, double m, double mx, double my, double mz) {
        v[i] = nc * m * R;
        if constexpr (GGA) {
            gx[i] = nc * (mx * R + m * dx * dR);
            gy[i] = nc * (my * R + m * dy * dR);
            gz[i] = nc * (mz * R + m * dz * dR);
        }
    };
    if (sh.l == 0) {
        put(0, 1.0, 1.0, 0.0, 0.0, 0.0);
        return 1;
    }
    if (sh.l == 1) {
        put(0, 1.0, dx, 1.0, 0.0, 0.0);
        put(1, 1.0, dy, 0.0, 1.0, 0.0);
        put(2, 1.0, dz, 0.0, 0.0, 1.0);
        return 3;
    }
    const double r3 = 1.7320508075688772;
    put(0, 1.0, dx * dx, 2.0 * dx, 0.0, 0.0);
    put(1, r3, dx * dy, dy, dx, 0.0);
    put(2, r3, dx * dz, dz, 0.0, dx);
    put(3, 1.0, dy * dy, 0.0, 2.0 * dy, 0.0);
    put(4, r3, dy * dz, 0.0, dz, dy);
    put(5, 1.0, dz * dz, 0.0, 0.0, 2.0 * dz);
    return 6;
}

// Phi of every shell for the two GEMMs (function-major, ld = ncols), from the same
// component values as the point kernel.
__global__ __launch_bounds__(256) void xc_collocate_kernel(const double* __restrict__ px,
                                                           const double* __restrict__ py,
                                                           const double* __restrict__ pz, int64_t ncols,
                                                           const ShellDev* __restrict__ shells,
                                                           const double* __restrict__ exps,
                                                           const double* __restrict__ coefs,
                                                           const int32_t* __restrict__ shell_row, int32_t nsh,
                                                           double* __restrict__ Phi)
{
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= ncols) return;
    const double x = px[col], y = py[col], z = pz[col];
    const int s0 = blockIdx.y * kXcShellsPerBlock;
    const int s1 = min(nsh, s0 + kXcShellsPerBlock);
    double v[6], unused[6];
    for (int si = s0; si < s1; ++si) {
        const ShellDev sh = shells[si];
        const int n = shell_values<false>(sh, exps, coefs, x - sh.x, y - sh.y, z - sh.z, v, unused, unused, unused);
        double* out = Phi + (int64_t)shell_row[si] * ncols + col;
        for (int i = 0; i < n; ++i) out[i * ncols] = v[i];
    }
}

// One lane per column of a launch over one or more tiles (a chunk of the unscreened build,
// or every tile of a batch group of the basis-screened build).  The basis values and
// gradients are recomputed from the shell data in both passes instead of being read from
// memory (a few exponentials per shell against four 8-byte loads per function): the kernel
// reads only F and writes G, whose rows follow the tile's shells.
template <bool GGA>
__global__ __launch_bounds__(256) void xc_point_kernel(const double* __restrict__ px, const double* __restrict__ py,
                                                       const double* __restrict__ pz, const double* __restrict__ pw,
                                                       const ShellDev* __restrict__ shells,
                                                       const double* __restrict__ exps,
                                                       const double* __restrict__ coefs,
                                                       const XcTile* __restrict__ tiles,
                                                       const int32_t* __restrict__ shell_cat, int32_t tile_batches,
                                                       const double* __restrict__ F, int64_t ncols, int fn,
                                                       double* __restrict__ G, double* __restrict__ epart)
{
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= ncols) return;
    const int tix = (int)(blockIdx.x / (unsigned)tile_batches);
    const XcTile t = tiles[tix];
    const int64_t lc = col - (int64_t)tix * tile_batches * kBatch;   // column within the tile
    const double* Ft = F + t.phi_off + lc;
    double* Gt = G + t.phi_off + lc;
    const double x = px[col], y = py[col], z = pz[col];
    double v[6], vx[6], vy[6], vz[6];
    double rho = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    int64_t row = 0;
    for (int si = 0; si < t.nsh; ++si) {
        const ShellDev sh = shells[shell_cat[t.sh_off + si]];
        const int n = shell_values<GGA>(sh, exps, coefs, x - sh.x, y - sh.y, z - sh.z, v, vx, vy, vz);
        for (int i = 0; i < n; ++i) {
            const double f = Ft[(row + i) * t.ncols];
            rho = fma(f, v[i], rho);
            if constexpr (GGA) {
                gx = fma(f, vx[i], gx);
                gy = fma(f, vy[i], gy);
                gz = fma(f, vz[i], gz);
            }
        }
        row += n;
    }
    gx *= 2.0;
    gy *= 2.0;
    gz *= 2.0;
    const double w = pw[col];
    XcVal e{0.0, 0.0, 0.0};
    if (rho >= kXcRhoMin) e = functional_eval(fn, rho, gx * gx + gy * gy + gz * gz);
    // G = 2 Z = w (E^rho Phi + 4 E^gamma grad rho . grad Phi)
    const double a = w * e.vr;
    const double b = 4.0 * w * e.vs;
    const double bx = b * gx, by = b * gy, bz = b * gz;
    row = 0;
    for (int si = 0; si < t.nsh; ++si) {
        const ShellDev sh = shells[shell_cat[t.sh_off + si]];
        const int n = shell_values<GGA>(sh, exps, coefs, x - sh.x, y - sh.y, z - sh.z, v, vx, vy, vz);
        for (int i = 0; i < n; ++i) {
            double g = a * v[i];
            if constexpr (GGA) g = fma(bx, vx[i], fma(by, vy[i], fma(bz, vz[i], g)));
            Gt[(row + i) * t.ncols] = g;
        }
        row += n;
    }
    epart[col] = w * e.e;
    epart[ncols + col] = w * rho;
}

// out[j] (+)= sum_i x[j * n + i], j = 0, 1: blocks of a fixed grid each write one partial in
// a fixed order; the last stage (one block) adds the partials to out (or overwrites it).
constexpr int kSumBlocks = 256;

__global__ __launch_bounds__(256) void xc_sum_kernel(const double* __restrict__ x, int64_t n,
                                                     double* __restrict__ partial)
{
    __shared__ double sh[2][256];
    for (int j = 0; j < 2; ++j) {
        double acc = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
            acc += x[j * n + i];
        sh[j][threadIdx.x] = acc;
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + h];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = sh[0][0];
        partial[kSumBlocks + blockIdx.x] = sh[1][0];
    }
}

__global__ __launch_bounds__(256) void xc_sum_final_kernel(const double* __restrict__ partial,
                                                           double* __restrict__ out, int accumulate)
{
    __shared__ double sh[2][256];
    sh[0][threadIdx.x] = partial[threadIdx.x];
    sh[1][threadIdx.x] = partial[kSumBlocks + threadIdx.x];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + h];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = (accumulate ? out[0] : 0.0) + sh[0][0];
        out[1] = (accumulate ? out[1] : 0.0) + sh[1][0];
    }
}

}  // namespace

hipError_t launch_xc_collocate(const double* px, const double* py, const double* pz, int64_t ncols,
                               const ShellDev* shells, const double* exps, const double* coefs,
                               const int32_t* shell_row, int32_t nsh, double* Phi, hipStream_t s)
{
    if (ncols <= 0 || nsh <= 0) return hipSuccess;
    dim3 grid((unsigned)((ncols + 255) / 256), (unsigned)((nsh + kXcShellsPerBlock - 1) / kXcShellsPerBlock));
    hipLaunchKernelGGL(xc_collocate_kernel, grid, dim3(256), 0, s, px, py, pz, ncols, shells, exps, coefs, shell_row,
                       nsh, Phi);
    return hipGetLastError();
}

hipError_t launch_xc_point(const double* px, const double* py, const double* pz, const double* pw, int64_t ncols,
                           const ShellDev* shells, const double* exps, const double* coefs, const XcTile* tiles,
                           const int32_t* shell_cat, int32_t tile_batches, const double* F, int fn, double* G,
                           double* epart, hipStream_t s)
{
    if (ncols <= 0) return hipSuccess;
    if (tile_batches < 1) return hipErrorInvalidValue;
    dim3 grid((unsigned)((ncols + 255) / 256));
    if (fn == SNK_XC_PBE)
        hipLaunchKernelGGL(xc_point_kernel<true>, grid, dim3(256), 0, s, px, py, pz, pw, shells, exps, coefs, tiles,
                           shell_cat, tile_batches, F, ncols, fn, G, epart);
    else
        hipLaunchKernelGGL(xc_point_kernel<false>, grid, dim3(256), 0, s, px, py, pz, pw, shells, exps, coefs, tiles,
                           shell_cat, tile_batches, F, ncols, fn, G, epart);
    return hipGetLastError();
}

hipError_t launch_xc_sum(const double* epart, int64_t n, double* partial, double* out, bool accumulate, hipStream_t s)
{
    hipLaunchKernelGGL(xc_sum_kernel, dim3(kSumBlocks), dim3(256), 0, s, epart, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(xc_sum_final_kernel, dim3(1), dim3(256), 0, s, partial, out, accumulate ? 1 : 0);
    return hipGetLastError();
}

}  // namespace snk
