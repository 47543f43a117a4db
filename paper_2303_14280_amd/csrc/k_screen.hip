// Density-dependent screening of the A.F step (Sec. II.E, the role of Eq. sp_set) with a
// rigorous block bound, on the GPU.
//
// A(r) is positive semi-definite (c^T A(r) c = int (sum_mu c_mu phi_mu)^2 / |r - r_i| >= 0),
// so |A_ab(r)| <= sqrt(A_aa(r) A_bb(r)).  For the energy contribution of the (A,B) shell-pair
// block over a batch j, e_AB = sum_i w_i F_A,i^T A_AB(r_i) F_B,i, Cauchy-Schwarz over the
// points gives |e_AB| <= U_A U_B with
//   U_A = sqrt( sum_i w_i ( sum_c |F_{A_c,i}| sqrt(A_{A_c A_c}(r_i)) )^2 ),
// which needs only the diagonal integrals (one same-shell pair per shell, evaluated in FP32
// with a 1% safety factor on U).  Skipping a set of blocks changes E_x by at most the sum of
// their U_A U_B.
//
// Per batch the builder bins log2(U) in half octaves, bounds the energy of every candidate
// skip set from the bin histogram (pairs in bins (k, l) have U_A U_B < 2^{(k+l+2)/2}),
// takes the largest skip set whose bound fits the batch's budget, and writes the surviving
// pairs as compacted run / B-task records for the A.F kernels.
//
// The learned screen refines this: the bound's survivors get a second estimate from the
// network (min of the bound and the prediction plus a margin; the bound alone for blocks
// whose features leave the training range), and a second half-octave histogram of these
// estimates spends the rest of the batch's budget.
#include "os3c.h"
#include "learn.h"

namespace snk {
namespace {

using namespace os3c;

constexpr int kNoBin = -100000;     // U == 0
constexpr int kGroup = 32;          // diagonal-bound shells per barrier
// The diagonal integrals are evaluated in FP32 (relative error ~1e-6 for these positive
// quantities); U is scaled by this factor so that it stays an upper bound.
constexpr double kBoundSafety = 1.01;

// ---------------------------------------------------------------------------------------
// U_A for the shells of one angular momentum L: one workgroup per batch, lane = point.
// With per-tile entry lists only the shells whose F rows the tile computed are evaluated;
// the caller has set U = 0 (and the features to their U = 0 values) for the others.
// Each wave evaluates kRed shells before it reduces their sums over its 64 lanes together.
// ---------------------------------------------------------------------------------------
constexpr int kRed = 8;

// Sums (MAX: maxima) over the 64 lanes of a wave of kRed per-lane values in 10 exchanges
// instead of 6 per value: each exchange halves the values a lane carries.  On return lane l
// holds the result for value l >> 3.
template <bool MAX>
__device__ __forceinline__ double wave_reduce8(const double (&v)[kRed], int lane)
{
    static_assert(kRed == 8, "three halving steps");
    auto op = [](double x, double y) { return MAX ? fmax(x, y) : x + y; };
    const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
    double w4[4], w2[2];
    sfor<0, 4>([&](auto jc) {
        constexpr int j = CV(jc);
        w4[j] = op(h5 ? v[j + 4] : v[j], __shfl_xor(h5 ? v[j] : v[j + 4], 32));
    });
    sfor<0, 2>([&](auto jc) {
        constexpr int j = CV(jc);
        w2[j] = op(h4 ? w4[j + 2] : w4[j], __shfl_xor(h4 ? w4[j] : w4[j + 2], 16));
    });
    double w1 = op(h3 ? w2[1] : w2[0], __shfl_xor(h3 ? w2[0] : w2[1], 8));
    w1 = op(w1, __shfl_xor(w1, 4));
    w1 = op(w1, __shfl_xor(w1, 2));
    return op(w1, __shfl_xor(w1, 1));
}

// The read-only arrays come as separate restrict-qualified arguments so that their uniform
// loads (entry indices, primitive-pair records) go through the scalar unit.
template <int L, typename TF>
__global__ __launch_bounds__(256) void diag_bound_kernel(DiagArgs a, const TF* __restrict__ F,
                                                         const PrimPair32* __restrict__ prims,
                                                         const int32_t* __restrict__ dsh,
                                                         const int32_t* __restrict__ drow,
                                                         const int32_t* __restrict__ dpb,
                                                         const int32_t* __restrict__ dnp,
                                                         const int32_t* __restrict__ dlist,
                                                         const int32_t* __restrict__ dcount)
{
    constexpr int N = ncart(L);
    __shared__ float tab[kBoysRows * kBoysCols];
    __shared__ double part[kGroup][4];
    __shared__ double npart[kGroup][4];
    __shared__ double mpart[kGroup][4];
    for (int i = threadIdx.x; i < kBoysRows * kBoysCols; i += blockDim.x) tab[i] = (float)a.tab[i];
    __syncthreads();
    const int batch = a.batch_order ? a.batch_order[blockIdx.x] : (int)blockIdx.x;
    const int64_t col = (int64_t)batch * kBatch + threadIdx.x;
    const float cx = (float)a.px[col], cy = (float)a.py[col], cz = (float)a.pz[col];
    const double w = a.pw[col], sw = sqrt(w);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tile = batch / a.tile_batches;
    const int32_t* list = dlist ? dlist + (int64_t)tile * a.n : nullptr;
    const int cnt = dlist ? dcount[tile] : a.n;
    const bool want_n = a.lun != nullptr, want_m = a.fmax != nullptr;
    // entries in groups of kGroup: per-wave partial sums in LDS, one barrier pair per group
    for (int s0 = 0; s0 < cnt; s0 += kGroup) {
        const int s1 = min(cnt, s0 + kGroup);
        for (int g0 = s0; g0 < s1; g0 += kRed) {
            double v[kRed], q[kRed], m[kRed];
            sfor<0, kRed>([&](auto jc) {
                constexpr int j = CV(jc);
                v[j] = 0.0;
                q[j] = 0.0;
                m[j] = 0.0;
                if (g0 + j < s1) {   // uniform over the workgroup
                    const int e = list ? list[g0 + j] : g0 + j;
                    float Acc[N];
                    diag_block<L, float>(prims + dpb[e], dnp[e], cx, cy, cz, tab, Acc);
                    const int row = drow[e];
                    double t = 0.0, f2 = 0.0, fm = 0.0;
                    sfor<0, N>([&](auto cc) {
                        constexpr int c = CV(cc);
                        const double f = cnorm(L, c) * (double)F[(int64_t)(row + c) * a.ld + col];
                        // A_cc of the unit-normalised component (FP32; U is scaled up by kBoundSafety)
                        t += fabs(f) * (double)sqrtf(fmaxf(Acc[c], 0.0f));
                        f2 += f * f;
                        fm = fmax(fm, fabs(f));
                    });
                    v[j] = w * t * t;
                    q[j] = w * f2;
                    m[j] = sw * fm;
                }
            });
            const double vs = wave_reduce8<false>(v, lane);
            const double qs = want_n ? wave_reduce8<false>(q, lane) : 0.0;
            const double ms = want_m ? wave_reduce8<true>(m, lane) : 0.0;
            const int j = lane >> 3;
            if ((lane & 7) == 0 && g0 + j < s1) {
                part[g0 - s0 + j][wave] = vs;
                npart[g0 - s0 + j][wave] = qs;
                mpart[g0 - s0 + j][wave] = ms;
            }
        }
        __syncthreads();
        if ((int)threadIdx.x < s1 - s0) {
            const int k = threadIdx.x;
            const int e = list ? list[s0 + k] : s0 + k;
            const int64_t o = (int64_t)batch * a.nshell + dsh[e];
            const double u = kBoundSafety * sqrt(part[k][0] + part[k][1] + part[k][2] + part[k][3]);
            a.U[o] = u;
            if (want_n)
                a.lun[o] = make_float2(learn::lg10(u),
                                       learn::lg10(sqrt(npart[k][0] + npart[k][1] + npart[k][2] + npart[k][3])));
            if (want_m) a.fmax[o] = fmax(fmax(mpart[k][0], mpart[k][1]), fmax(mpart[k][2], mpart[k][3]));
        }
        __syncthreads();
    }
}

// One workgroup per (tile, angular momentum): each thread takes a contiguous run of the
// diagonal entries, counts those whose shell the tile flags, and after a workgroup scan
// writes their indices in ascending order.
__global__ __launch_bounds__(256) void diag_lists_kernel(DiagLists d, const int32_t* __restrict__ flag,
                                                         int32_t nshell)
{
    __shared__ int32_t part[256];
    const int t = blockIdx.x, l = blockIdx.y, tid = threadIdx.x;
    const int n = d.n[l];
    const int32_t* f = flag + (int64_t)t * nshell;
    const int32_t* dsh = d.dsh[l];
    const int per = (n + 255) / 256;
    const int k0 = min(n, tid * per), k1 = min(n, k0 + per);
    int cnt = 0;
    for (int k = k0; k < k1; ++k) cnt += f[dsh[k]] != 0;
    part[tid] = cnt;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int v = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int r = part[tid] - cnt;
    int32_t* out = d.list[l] + (int64_t)t * n;
    for (int k = k0; k < k1; ++k)
        if (f[dsh[k]]) out[r++] = k;
    if (tid == 255) d.count[l][t] = part[255];
}

// block-wide exclusive prefix count of a per-thread flag (256 threads), returns the total
__device__ __forceinline__ int block_scan_flag(bool flag, int* wsum, int* rank)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long m = __ballot(flag);
    const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int in_wave = __popcll(m & lt);
    if (lane == 0) wsum[wave] = __popcll(m);
    __syncthreads();
    int before = 0;
    for (int k = 0; k < wave; ++k) before += wsum[k];
    const int total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    *rank = before + in_wave;
    return total;
}

__device__ __forceinline__ int64_t pair_index(int s, int t)
{
    if (s < t) {
        const int x = s;
        s = t;
        t = x;
    }
    return (int64_t)s * (s + 1) / 2 + t;
}

// ---------------------------------------------------------------------------------------
// Bound set-up shared by the list builder and the learned estimate pass: per-shell bins of
// log2 U, the batch's bound threshold S (pairs with bins[A] + bins[B] < S are skipped), the
// bound on their energy, and the shells that can pair above S, grouped by l in shell order.
// ---------------------------------------------------------------------------------------
struct BoundShared {
    int32_t hist[kNBins];
    union {
        double cnt_s[2 * kNBins];      // bound set-up: pair counts per bin sum
        int32_t queue[4 * kNBins];     // learned estimate, afterwards: candidate queue
    };
    int32_t aoff[4];
    int32_t S, S2, bmin, bmax;
    double acc;
    int wsum[4];
    long long wsum64[4];
    int carry;
};

// Shells per l packed into one 64-bit counter (21 bits per angular momentum)
constexpr int kLBits = 21;

__device__ void bound_setup(const double* __restrict__ Ub, int nshell, const int32_t* __restrict__ shell_l,
                            double eps, double eps_low, int32_t* bins, int32_t* act, BoundShared& sh,
                            bool all_active = false)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int k = tid; k < kNBins; k += blockDim.x) sh.hist[k] = 0;
    if (tid == 0) {
        sh.bmin = kNBins;
        sh.bmax = -1;
    }
    __syncthreads();
    int lo = kNBins, hi = -1;
    for (int s = tid; s < nshell; s += blockDim.x) {
        const double u = Ub[s];
        int b = kNoBin;
        if (u > 0.0) {
            b = (int)floor(2.0 * log2(u)) + kBinOff;
            b = b < 0 ? 0 : (b >= kNBins ? kNBins - 1 : b);   // clamped: still an upper bin
            atomicAdd(&sh.hist[b], 1);
            lo = min(lo, b);
            hi = max(hi, b);
        }
        bins[s] = b;
    }
    if (hi >= 0) {
        atomicMin(&sh.bmin, lo);
        atomicMax(&sh.bmax, hi);
    }
    __syncthreads();
    // the histogram is empty outside [bmin, bmax]: only bin sums 2 bmin .. 2 bmax can be non-zero
    const int bmin = sh.bmin, bmax = sh.bmax;
    // unordered pairs per bin sum s = k + l (index space), weighted by the pair bound (integer
    // counts, exact in any order)
    for (int s = 2 * bmin + tid; s <= 2 * bmax; s += blockDim.x) {
        double c = 0.0;
        const int k0 = max(bmin, s - bmax), k1 = min(bmax, s - bmin);
        for (int k = k0; k <= k1; ++k) c += (double)sh.hist[k] * (double)sh.hist[s - k];
        if ((s & 1) == 0) c += (double)sh.hist[s >> 1];
        sh.cnt_s[s] = 0.5 * c;
    }
    __syncthreads();
    if (tid == 0) {
        // largest S with sum_{s < S} count(s) * 2^{(s - 2 kBinOff + 2)/2} <= eps (bin sums with
        // no pairs extend S; past 2 bmax every sum is empty)
        double acc = 0.0;
        int S = 1 << 30, S2 = 1 << 30;   // every U is zero: nothing to evaluate
        if (bmax >= 0) {
            S = 2 * kNBins;
            for (int s = 2 * bmin; s <= 2 * bmax; ++s) {
                const double cs = sh.cnt_s[s];
                if (cs == 0.0) continue;
                const double add = cs * exp2(0.5 * (double)(s - 2 * kBinOff + 2));
                if (acc + add > eps) {
                    S = s;
                    break;
                }
                acc += add;
            }
            // bound pairs S .. S2-1 may go to FP32 within eps_low
            S2 = 2 * kNBins;
            double low = 0.0;
            for (int s = S; s <= 2 * bmax; ++s) {
                const double add = sh.cnt_s[s] * exp2(0.5 * (double)(s - 2 * kBinOff + 2));
                if (low + add > eps_low) {
                    S2 = s;
                    break;
                }
                low += add;
            }
        }
        sh.S = S;
        sh.S2 = S2;
        sh.acc = acc;
        sh.aoff[0] = 0;
    }
    __syncthreads();
    // Shells that can pair above S, by l in ascending shell order: each thread takes a
    // contiguous run of shells, counts its shells per l, and places them after an exclusive
    // scan of the packed counts over the workgroup.
    const int S = sh.S;
    const int per = (nshell + (int)blockDim.x - 1) / (int)blockDim.x;
    const int s0 = min(nshell, tid * per), s1 = min(nshell, s0 + per);
    auto active = [&](int s) { return all_active || (bins[s] != kNoBin && bins[s] + bmax >= S); };
    long long mine = 0;
    for (int s = s0; s < s1; ++s)
        if (active(s)) mine += 1ll << (kLBits * shell_l[s]);
    long long incl = mine;
    for (int o = 1; o < 64; o <<= 1) {
        const long long v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    if (lane == 63) sh.wsum64[wave] = incl;
    __syncthreads();
    long long before = incl - mine;
    for (int w = 0; w < wave; ++w) before += sh.wsum64[w];
    const long long total = sh.wsum64[0] + sh.wsum64[1] + sh.wsum64[2] + sh.wsum64[3];
    constexpr long long kMask = (1ll << kLBits) - 1;
    const int n0 = (int)(total & kMask), n1 = (int)((total >> kLBits) & kMask);
    const int n2 = (int)((total >> (2 * kLBits)) & kMask);
    int p0 = (int)(before & kMask), p1 = n0 + (int)((before >> kLBits) & kMask);
    int p2 = n0 + n1 + (int)((before >> (2 * kLBits)) & kMask);
    for (int s = s0; s < s1; ++s)
        if (active(s)) {
            const int l = shell_l[s];
            if (l == 0) act[p0++] = s;
            else if (l == 1) act[p1++] = s;
            else act[p2++] = s;
        }
    if (tid == 0) {
        sh.aoff[1] = n0;
        sh.aoff[2] = n0 + n1;
        sh.aoff[3] = n0 + n1 + n2;
    }
    __syncthreads();
}

__device__ __forceinline__ int est_bin(float lest)
{
    if (!(lest > -1e30f)) return -1;            // zero estimate
    int b = (int)floorf(2.0f * lest) + kBinOff;
    return b < 0 ? 0 : (b >= kNBins ? kNBins - 1 : b);
}

// ---------------------------------------------------------------------------------------
// Learned estimate pass: one workgroup per batch; each wave takes 16 candidate pairs at a
// time and runs the network on them in one sweep of matrix-core ops.
// Dynamic shared memory: bins[nshell] + active[nshell] (int32).
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void screen_est_kernel(EstArgs a)
{
    extern __shared__ int32_t dyn[];
    int32_t* bins = dyn;
    int32_t* act = dyn + a.nshell;
    __shared__ BoundShared sh;
    __shared__ int32_t lhist[kNBins];

    const int batch = a.batch_order ? a.batch_order[blockIdx.x] : (int)blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    const double* Ub = a.U + (int64_t)batch * a.nshell;
    const float2* Lb = a.lun + (int64_t)batch * a.nshell;
    __shared__ int32_t lmin, lmax;
    for (int k = tid; k < kNBins; k += blockDim.x) lhist[k] = 0;
    if (tid == 0) {
        lmin = kNBins;
        lmax = -1;
    }
    int elo = kNBins, ehi = -1;   // this thread's range of estimate bins
    bound_setup(Ub, a.nshell, a.shell_l, a.eps_batch, 0.0, bins, act, sh);
    const int S = sh.S;
    const BatchGeo bg = a.geo[batch];

    __shared__ __align__(16) learn::MlpShared msh;
    learn::MlpRegs R;
    learn::load_mlp(a.params, a.norm, a.lo, a.hi, R, msh);
    const float log2_10 = 3.32192809488736f;
    const float mlog2 = a.margin * log2_10;

    // Candidates, enumerated one of two ways (uniform per batch): the static list of pairs
    // with kept primitive pairs (class order, consecutive records) when most pairs are
    // active, or the combinations of the shells the bound leaves active (same-l classes over
    // the triangle ai >= bi; the active lists ascend in shell index) when few are.  Pairs
    // the bound already skips on this batch are dropped either way.
    //
    // In rounds of kQueue candidates: the whole workgroup applies the bound's test (one
    // candidate per thread) and queues the survivors' positions k in the list of pairs with
    // kept primitive pairs; then the waves run the network on the queue, 16 entries at a time.
    // Every survivor's estimate lands at its own k and the histogram counts are sums of
    // integers, so the queue's order does not change the result.
    __shared__ int64_t coff[7];
    __shared__ int use_list;
    __shared__ int qn;
    constexpr int kQueue = 4 * kNBins;
    int32_t* queue = sh.queue;   // the bin-sum counts' space, free once the bound is set up
    if (tid == 0) {
        int64_t acc = 0;
        for (int c = 0; c < 6; ++c) {
            const int la = kClassLA_dev(c), lb = kClassLB_dev(c);
            const int64_t nA = sh.aoff[la + 1] - sh.aoff[la], nB = sh.aoff[lb + 1] - sh.aoff[lb];
            coff[c] = acc;
            acc += la == lb ? nA * (nA + 1) / 2 : nA * nB;
        }
        coff[6] = acc;
        use_list = 2 * acc >= a.nne;
    }
    __syncthreads();
    const bool list = use_list != 0;
    const int64_t total = list ? a.nne : coff[6];
    // the bound's test of candidate i: its position k, or -1
    auto survivor = [&](int64_t i) -> int32_t {
        int aa, b;
        int32_t k;
        if (list) {
            const int2 ab = a.ne_ab[i];
            aa = ab.x;
            b = ab.y;
            k = (int32_t)i;
        } else {
            int c = 0;
            while (c < 5 && i >= coff[c + 1]) ++c;
            const int la = kClassLA_dev(c), lb = kClassLB_dev(c);
            const int64_t j = i - coff[c];
            int ai, bi;
            if (la == lb) {
                ai = (int)((sqrtf(8.0f * (float)j + 1.0f) - 1.0f) * 0.5f);
                while ((int64_t)ai * (ai + 1) / 2 > j) --ai;
                while ((int64_t)(ai + 1) * (ai + 2) / 2 <= j) ++ai;
                bi = (int)(j - (int64_t)ai * (ai + 1) / 2);
            } else {
                const int nB = sh.aoff[lb + 1] - sh.aoff[lb];
                ai = (int)(j / nB);
                bi = (int)(j - (int64_t)ai * nB);
            }
            aa = act[sh.aoff[la] + ai];
            b = act[sh.aoff[lb] + bi];
            k = -1;
        }
        if (bins[aa] == kNoBin || bins[b] == kNoBin || bins[aa] + bins[b] < S) return -1;
        return list ? k : a.ne_pos[pair_index(aa, b)];
    };
    struct Cand {
        bool valid;
        int32_t k;
        PairFeat pf;
        float lp;
        float2 ua, ub;
    };
    auto fetch = [&](int idx, int n, Cand& d) {
        d.valid = idx < n;
        if (d.valid) {
            d.k = queue[idx];
            const int2 ab = a.ne_ab[d.k];
            d.pf = a.ne_feat[d.k];
            d.lp = a.ne_lp[d.k];
            d.ua = Lb[ab.x];
            d.ub = Lb[ab.y];
        } else {
            d.k = 0;
            d.pf = PairFeat{};
            d.lp = 0.0f;
            d.ua = d.ub = make_float2(0.0f, 0.0f);
        }
    };

    for (int64_t base = 0; base < total; base += kQueue) {
        if (tid == 0) qn = 0;
        __syncthreads();
        const int64_t end = base + kQueue < total ? base + kQueue : total;
        for (int64_t i = base + tid; i < end; i += blockDim.x) {
            const int32_t k = survivor(i);
            if (k >= 0) queue[atomicAdd(&qn, 1)] = k;
        }
        __syncthreads();
        const int n = qn;
        Cand cur, nxt;
        int q = wave * 16;
        fetch(q + r, n, nxt);
        for (; q < n; q += 64) {
            cur = nxt;
            fetch(q + 64 + r, n, nxt);
            float f[16];
            learn::block_features(cur.pf, cur.lp, bg, cur.ua.x, cur.ub.x, cur.ua.y, cur.ub.y, f);
            float x[4];
            bool oob = false;
            for (int e = 0; e < 4; ++e) {
                // this lane supplies features 4g .. 4g+3 (constant-index selects, no scratch)
                float v = f[e];
                v = g == 1 ? f[4 + e] : v;
                v = g == 2 ? f[8 + e] : v;
                v = g == 3 ? f[12 + e] : v;
                x[e] = v;
                oob |= !(v >= msh.lo[4 * g + e] && v <= msh.hi[4 * g + e]);
            }
            const unsigned long long mo = __ballot(oob);
            const bool sample_oob = ((mo >> r) & 0x0001000100010001ull) != 0ull;
            const float y = learn::mlp_eval16(R, msh, x);
            if (g == 0 && cur.valid) {
                // log2 of the bound c_AB U_A U_B (an over-estimate where a factor was clamped)
                const float lbeta = (learn::log_cab(cur.pf) + cur.ua.x + cur.ub.x) * log2_10;
                const float lest = sample_oob ? lbeta : fminf(lbeta, fmaf(y, log2_10, mlog2));
                const int64_t o = (int64_t)batch * a.nne + cur.k;
                a.est[o] = lest;
                if (a.yraw) a.yraw[o] = y;
                const int eb = est_bin(lest);
                if (eb >= 0) {
                    atomicAdd(&lhist[eb], 1);
                    elo = min(elo, eb);
                    ehi = max(ehi, eb);
                }
            }
        }
        __syncthreads();   // the queue is refilled
    }
    if (ehi >= 0) {
        atomicMin(&lmin, elo);
        atomicMax(&lmax, ehi);
    }
    __syncthreads();
    if (tid == 0) {
        // largest T with sum_{k < T} count(k) 2^{(k + 1 - kBinOff)/2} <= budget left by the bound
        // (empty bins extend T; the histogram is empty outside [lmin, lmax])
        const double rem = a.eps_batch - sh.acc;
        double acc = 0.0;
        int T = kNBins, T2 = kNBins;
        if (lmax >= 0) {
            for (int k = lmin; k <= lmax; ++k) {
                if (lhist[k] == 0) continue;
                const double add = (double)lhist[k] * exp2(0.5 * (double)(k + 1 - kBinOff));
                if (acc + add > rem) {
                    T = k;
                    break;
                }
                acc += add;
            }
            // then the FP32 set: bins T .. T2-1 whose estimates sum to at most eps_low
            double low = 0.0;
            for (int k = T; k <= lmax; ++k) {
                const double add = (double)lhist[k] * exp2(0.5 * (double)(k + 1 - kBinOff));
                if (low + add > a.eps_low) {
                    T2 = k;
                    break;
                }
                low += add;
            }
        }
        a.thr[batch] = T;
        a.thr2[batch] = T2;
        a.skipped[batch] = sh.acc + acc;
    }
}

// ---------------------------------------------------------------------------------------
// List builder.  WRITE = false: counts only; WRITE = true: records at the scanned offsets.
// Dynamic shared memory: bins[nshell] + active[nshell] + tilecnt[nshell] (int32).
// ---------------------------------------------------------------------------------------
template <bool WRITE>
__global__ __launch_bounds__(256) void screen_kernel(ScreenArgs a)
{
    extern __shared__ int32_t dyn[];
    int32_t* bins = dyn;
    int32_t* act = dyn + a.nshell;
    int32_t* tilecnt = dyn + 2 * a.nshell;
    __shared__ BoundShared sh;

    const int batch = a.batch_order ? a.batch_order[blockIdx.x] : (int)blockIdx.x;
    const int tid = threadIdx.x;
    const double* Ub = a.U + (int64_t)batch * a.nshell;
    const bool learned = a.est != nullptr;
    // the paper's selection decides every pair itself (Eq. sp_set), without the bound's bins
    bound_setup(Ub, a.nshell, a.shell_l, a.eps_batch, learned ? 0.0 : a.eps_low, bins, act, sh, a.link != 0);
    const int S = sh.S, S2 = sh.S2;
    const int T = learned ? a.thr[batch] : 0;
    const int T2 = learned ? a.thr2[batch] : 0;
    const float* estb = learned ? a.est + (int64_t)batch * a.nne : nullptr;
    // block (aa, b) of the batch is evaluated in list category cat (0: FP64 or all, 1: FP32)
    int cat = 0;
    const double* fm = a.link ? a.fmax + (int64_t)batch * a.nshell : nullptr;
    const double phit = a.link ? a.phit[batch] : 0.0;
    // Eq. sp_set: the energy estimate or the exchange-matrix estimate reaches the threshold
    auto link_keep = [&](int aa, int b, int64_t p) -> bool {
        const double at = a.atil[p];
        return fm[aa] * fm[b] * at >= a.link_eps || ::fmax(fm[aa], fm[b]) * phit * at >= a.link_eps;
    };
    // The learned estimate never exceeds the bound c_AB U_A U_B it was given (U clamped below at
    // 1e-40 there), whose bin lies below fb(A) + fb(B) - kBinOff + 2 with fb = max(bin, the bin of
    // 1e-40); so with T > 0 a pair whose bins sum to at most T + kBinOff - 3 cannot reach bin T,
    // and is dropped without reading its estimate.
    constexpr int kLunFloorBin = kBinOff - 266;   // floor(2 log2 1e-40) + kBinOff
    const int tcut = T + kBinOff - 3;
    auto keep = [&](int aa, int b) -> bool {
        if (!a.link && bins[aa] + bins[b] < S) return false;
        if (learned && T > 0 && max(bins[aa], kLunFloorBin) + max(bins[b], kLunFloorBin) <= tcut) return false;
        const int64_t p = pair_index(aa, b);
        const int32_t pos = a.ne_pos[p];   // a 4-byte table instead of the pair record
        if (pos < 0) return false;
        if (a.link && !link_keep(aa, b, p)) return false;
        bool high = true;
        if (learned) {
            const int eb = est_bin(estb[pos]);
            if (eb < T) return false;
            high = eb >= T2;
        } else {
            high = bins[aa] + bins[b] >= S2;
        }
        return a.nlist == 6 || (cat == 0) == high;
    };

    for (int c = 0; c < a.nlist; ++c) {
        cat = c / 6;
        const int cl = c % 6;
        const int la = kClassLA_dev(cl), lb = kClassLB_dev(cl), TA = kListTile(c);
        const int nA = sh.aoff[la + 1] - sh.aoff[la], nB = sh.aoff[lb + 1] - sh.aoff[lb];
        const int32_t* actA = act + sh.aoff[la];
        const int32_t* actB = act + sh.aoff[lb];
        const int nt = (nA + TA - 1) / TA;
        const int64_t ncombo = (int64_t)nt * nB;
        for (int t = tid; t < nt; t += blockDim.x) tilecnt[t] = 0;
        if (tid == 0) sh.carry = 0;
        __syncthreads();
        int64_t npair = 0;
        double lskip = 0.0;   // link mode: bound on the energy of the blocks it drops
        // pass 1: per-tile counts
        for (int64_t i0 = 0; i0 < ncombo; i0 += blockDim.x) {
            const int64_t i = i0 + tid;
            int mask = 0;
            if (i < ncombo) {
                const int t = (int)(i / nB), bi = (int)(i - (int64_t)t * nB);
                const int b = actB[bi];
                for (int k = 0; k < TA; ++k) {
                    const int ai = t * TA + k;
                    if (ai >= nA) break;
                    const int aa = actA[ai];
                    if (la == lb && aa < b) continue;
                    if (!keep(aa, b)) {
                        if (!WRITE && a.link && cat == 0) {
                            const int64_t p = pair_index(aa, b);
                            if (a.ne_pos[p] >= 0 && !link_keep(aa, b, p))
                                lskip += (aa == b ? 0.5 : 1.0) * Ub[aa] * Ub[b];
                        }
                        continue;
                    }
                    mask |= 1 << k;
                    if (!WRITE && a.shell_flag) {
                        // both shells receive G contributions (idempotent flag stores)
                        int32_t* f = a.shell_flag + (int64_t)(batch / a.tile_batches) * a.nshell;
                        f[aa] = 1;
                        f[b] = 1;
                    }
                }
                if (mask) {
                    atomicAdd(&tilecnt[t], 1);
                    npair += __popc(mask);
                }
            }
        }
        __syncthreads();
        if (!WRITE) {
            // reduce npair, the link-skipped bound and the run and B-task counts over the block
            // (integer counts; the bound sums in a fixed order)
            int nrun = 0, nbt = 0;
            for (int t = tid; t < nt; t += blockDim.x) {
                const int n = tilecnt[t];
                nbt += n;
                nrun += n > 0;
            }
            double v = (double)npair, ls = lskip;
            for (int o = 32; o > 0; o >>= 1) {
                v += __shfl_xor(v, o);
                ls += __shfl_xor(ls, o);
                nrun += __shfl_xor(nrun, o);
                nbt += __shfl_xor(nbt, o);
            }
            __shared__ double red[4], lred[4];
            __shared__ int rred[4], bred[4];
            if ((tid & 63) == 0) {
                red[tid >> 6] = v;
                lred[tid >> 6] = ls;
                rred[tid >> 6] = nrun;
                bred[tid >> 6] = nbt;
            }
            __syncthreads();
            if (tid == 0) {
                if (a.link) sh.acc += lred[0] + lred[1] + lred[2] + lred[3];
                a.counts[((int64_t)batch * a.nlist + c) * 2] = rred[0] + rred[1] + rred[2] + rred[3];
                a.counts[((int64_t)batch * a.nlist + c) * 2 + 1] = bred[0] + bred[1] + bred[2] + bred[3];
                a.npairs[(int64_t)batch * a.nlist + c] = (int64_t)(red[0] + red[1] + red[2] + red[3]);
            }
            __syncthreads();
            continue;
        }
        // WRITE: run records from an exclusive scan of the tile counts, 256 tiles at a time
        // (runs and B tasks counted together in one 64-bit value: runs << 32 | B tasks)
        {
            const int64_t rb = a.run_base[(int64_t)c * (a.nbatch + 1) + batch];
            const int64_t bb = a.bt_base[(int64_t)c * (a.nbatch + 1) + batch];
            const int RS = 2 + TA;
            const int lane = tid & 63, wave = tid >> 6;
            long long carry = 0;
            for (int t0 = 0; t0 < nt; t0 += blockDim.x) {
                const int t = t0 + tid;
                const int n = t < nt ? tilecnt[t] : 0;
                const long long mine = n > 0 ? (1ll << 32) + n : 0ll;
                long long incl = mine;
                for (int o = 1; o < 64; o <<= 1) {
                    const long long x = __shfl_up(incl, o);
                    if (lane >= o) incl += x;
                }
                if (lane == 63) sh.wsum64[wave] = incl;
                __syncthreads();
                long long before = carry + incl - mine;
                for (int w = 0; w < wave; ++w) before += sh.wsum64[w];
                const long long tot = sh.wsum64[0] + sh.wsum64[1] + sh.wsum64[2] + sh.wsum64[3];
                if (n > 0) {
                    const int64_t r = rb + (before >> 32), bt = bb + (before & 0xffffffffll);
                    int32_t* rec = a.runs[c] + r * RS;
                    rec[0] = (int32_t)bt;
                    rec[1] = (int32_t)(bt + n);
                    for (int k = 0; k < TA; ++k) {
                        const int ai = t * TA + k;
                        rec[2 + k] = ai < nA ? a.shell_row[actA[ai]] : -1;
                    }
                }
                carry += tot;
                __syncthreads();   // wsum64 is reused
            }
            if (tid == 0) {
                a.batch_run_off[c][batch] = (int32_t)rb;
                if (batch == a.nbatch - 1) a.batch_run_off[c][a.nbatch] = (int32_t)(rb + (carry >> 32));
            }
            if (tid == 0) sh.carry = 0;
            __syncthreads();
        }
        // pass 2: B-task records in (tile, B) order
        const int64_t bb = a.bt_base[(int64_t)c * (a.nbatch + 1) + batch];
        const int BS = 2 + 2 * TA;
        for (int64_t i0 = 0; i0 < ncombo; i0 += blockDim.x) {
            const int64_t i = i0 + tid;
            int mask = 0;
            int t = 0, b = 0;
            if (i < ncombo) {
                t = (int)(i / nB);
                b = actB[(int)(i - (int64_t)t * nB)];
                for (int k = 0; k < TA; ++k) {
                    const int ai = t * TA + k;
                    if (ai >= nA) break;
                    const int aa = actA[ai];
                    if (la == lb && aa < b) continue;
                    if (!keep(aa, b)) continue;
                    mask |= 1 << k;
                }
            }
            int rank;
            const int tot = block_scan_flag(mask != 0, sh.wsum, &rank);
            if (mask) {
                const int64_t slot = bb + sh.carry + rank;
                int32_t* rec = a.btasks[c] + slot * BS;
                rec[0] = a.shell_row[b];
                rec[1] = mask;
                for (int k = 0; k < TA; ++k) {
                    const int ai = t * TA + k;
                    int pb = 0, np = 0;
                    if (mask & (1 << k)) {
                        const PairHdr& h = a.pairs[pair_index(actA[ai], b)];
                        pb = h.prim_begin;
                        np = h.nprim;
                    }
                    rec[2 + 2 * k] = pb;
                    rec[3 + 2 * k] = np;
                }
            }
            __syncthreads();
            if (tid == 0) sh.carry += tot;
            __syncthreads();
        }
    }
    if (!WRITE && !learned && tid == 0) a.skipped[batch] = sh.acc;
}

// exclusive scans of the per-(batch, class) counts: run_base / bt_base [6][nbatch+1].
// One workgroup per class; thread t scans a contiguous segment of batches, the segment
// totals are scanned in LDS (fixed order, integer sums).
__global__ __launch_bounds__(256) void screen_scan_kernel(const int32_t* __restrict__ counts, int32_t nbatch,
                                                          int32_t nlist, int64_t* __restrict__ run_base,
                                                          int64_t* __restrict__ bt_base)
{
    __shared__ int64_t sr[256], sb[256];
    const int c = blockIdx.x, t = threadIdx.x;
    const int seg = (nbatch + 255) / 256;
    const int j0 = min(nbatch, t * seg), j1 = min(nbatch, j0 + seg);
    int64_t r = 0, b = 0;
    for (int j = j0; j < j1; ++j) {
        r += counts[((int64_t)j * nlist + c) * 2];
        b += counts[((int64_t)j * nlist + c) * 2 + 1];
    }
    sr[t] = r;
    sb[t] = b;
    __syncthreads();
    if (t == 0) {
        int64_t ar = 0, ab = 0;
        for (int k = 0; k < 256; ++k) {
            const int64_t xr = sr[k], xb = sb[k];
            sr[k] = ar;
            sb[k] = ab;
            ar += xr;
            ab += xb;
        }
        run_base[(int64_t)c * (nbatch + 1) + nbatch] = ar;
        bt_base[(int64_t)c * (nbatch + 1) + nbatch] = ab;
    }
    __syncthreads();
    r = sr[t];
    b = sb[t];
    for (int j = j0; j < j1; ++j) {
        run_base[(int64_t)c * (nbatch + 1) + j] = r;
        bt_base[(int64_t)c * (nbatch + 1) + j] = b;
        r += counts[((int64_t)j * nlist + c) * 2];
        b += counts[((int64_t)j * nlist + c) * 2 + 1];
    }
}

}  // namespace

hipError_t launch_diag_bound(int l, const DiagArgs& a, hipStream_t s)
{
    if (a.list && (a.tile_batches < 1 || !a.count)) return hipErrorInvalidValue;
    if (a.nbatch <= 0 || a.n <= 0) return hipSuccess;
    DiagArgs b = a;
    if (!b.list) b.tile_batches = 1;   // unused, but keeps the tile index defined
    dim3 grid(a.nbatch), block(kBatch);
#define SNK_DB(L)                                                                                                  \
    if (a.F32)                                                                                                     \
        hipLaunchKernelGGL((diag_bound_kernel<L, float>), grid, block, 0, s, b, a.F32, a.prims, a.dsh, a.drow,     \
                           a.dpb, a.dnp, a.list, a.count);                                                         \
    else                                                                                                           \
        hipLaunchKernelGGL((diag_bound_kernel<L, double>), grid, block, 0, s, b, a.F, a.prims, a.dsh, a.drow,      \
                           a.dpb, a.dnp, a.list, a.count)
    switch (l) {
        case 0: SNK_DB(0); break;
        case 1: SNK_DB(1); break;
        case 2: SNK_DB(2); break;
        default: return hipErrorInvalidValue;
    }
#undef SNK_DB
    return hipGetLastError();
}

hipError_t launch_diag_lists(const DiagLists& d, const int32_t* flag, int32_t ntile, int32_t nshell, hipStream_t s)
{
    if (ntile <= 0) return hipSuccess;
    for (int l = 0; l < 3; ++l)
        if (!d.count[l] || (d.n[l] > 0 && (!d.list[l] || !d.dsh[l]))) return hipErrorInvalidValue;
    hipLaunchKernelGGL(diag_lists_kernel, dim3(ntile, 3), dim3(256), 0, s, d, flag, nshell);
    return hipGetLastError();
}

hipError_t launch_screen(bool write, const ScreenArgs& a, hipStream_t s)
{
    if (a.nbatch <= 0) return hipSuccess;
    const size_t shm = (size_t)3 * a.nshell * sizeof(int32_t);
    if (write)
        hipLaunchKernelGGL((screen_kernel<true>), dim3(a.nbatch), dim3(256), shm, s, a);
    else
        hipLaunchKernelGGL((screen_kernel<false>), dim3(a.nbatch), dim3(256), shm, s, a);
    return hipGetLastError();
}

// One workgroup per tile: each thread takes a contiguous run of shells, counts the functions
// of its flagged shells, and after a workgroup exclusive scan writes their row indices.
__global__ __launch_bounds__(256) void tile_rows_kernel(const int32_t* __restrict__ flag, int32_t nshell,
                                                        const int32_t* __restrict__ shell_l,
                                                        const int32_t* __restrict__ shell_row, int32_t nbf,
                                                        int32_t* __restrict__ rows, int32_t* __restrict__ count)
{
    __shared__ int32_t part[256];
    const int tile = blockIdx.x, tid = threadIdx.x;
    const int32_t* f = flag + (int64_t)tile * nshell;
    const int per = (nshell + 255) / 256;
    const int s0 = min(nshell, tid * per), s1 = min(nshell, s0 + per);
    int n = 0;
    for (int sh = s0; sh < s1; ++sh)
        if (f[sh]) n += (shell_l[sh] + 1) * (shell_l[sh] + 2) / 2;
    part[tid] = n;
    __syncthreads();
    // Hillis-Steele inclusive scan over the 256 partial counts
    for (int o = 1; o < 256; o <<= 1) {
        const int v = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int r = part[tid] - n;
    int32_t* out = rows + (int64_t)tile * nbf;
    for (int sh = s0; sh < s1; ++sh) {
        if (!f[sh]) continue;
        const int nf = (shell_l[sh] + 1) * (shell_l[sh] + 2) / 2;
        for (int k = 0; k < nf; ++k) out[r++] = shell_row[sh] + k;
    }
    if (tid == 255) count[tile] = part[255];
}

hipError_t launch_tile_rows(const int32_t* shell_flag, int32_t ntile, int32_t nshell, const int32_t* shell_l,
                            const int32_t* shell_row, int32_t nbf, int32_t* rows, int32_t* count, hipStream_t s)
{
    if (ntile <= 0) return hipSuccess;
    if (!shell_flag || !shell_l || !shell_row || !rows || !count) return hipErrorInvalidValue;
    hipLaunchKernelGGL(tile_rows_kernel, dim3(ntile), dim3(256), 0, s, shell_flag, nshell, shell_l, shell_row, nbf,
                       rows, count);
    return hipGetLastError();
}

// One workgroup per batch of a group, lane = point: phit[b] = max_i sqrt(w_i) sum_mu |Phi_mu,i|
// over the rows of the batch's tile (the paper's phi-tilde of the sn-LinK estimates).
template <typename T>
__global__ __launch_bounds__(256) void phisum_kernel(const T* __restrict__ Phi, const int32_t* __restrict__ roff,
                                                     int32_t ntile, int32_t tile_batches, int64_t ncols_last,
                                                     const double* __restrict__ pw, double* __restrict__ phit)
{
    __shared__ double red[4];
    const int b = blockIdx.x;
    const int t = b / tile_batches;
    const int64_t tile_cols = (int64_t)tile_batches * kBatch;
    const int64_t ncols = t == ntile - 1 ? ncols_last : tile_cols;
    const T* base = Phi + (int64_t)roff[t] * tile_cols;   // every tile before t is full
    const int64_t c = (int64_t)(b - t * tile_batches) * kBatch + threadIdx.x;
    double v = 0.0;
    for (int r = roff[t]; r < roff[t + 1]; ++r) v += fabs((double)base[(int64_t)(r - roff[t]) * ncols + c]);
    v *= sqrt(pw[(int64_t)b * kBatch + threadIdx.x]);
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) phit[b] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// One workgroup per batch b of a group, one wave per row k of the batch's tile:
// out[b][k] = max_i sqrt(w_i) |Phi_k,i| over the batch's points (the Phi-tilde of the sn-LinK
// estimates; rows beyond the tile's nB up to ld are left untouched).
template <typename T>
__global__ __launch_bounds__(256) void phimax_kernel(const T* __restrict__ Phi, const int32_t* __restrict__ roff,
                                                     int32_t ntile, int32_t tile_batches, int64_t ncols_last,
                                                     const double* __restrict__ pw, double* __restrict__ out,
                                                     int64_t ld)
{
    const int b = blockIdx.x;
    const int t = b / tile_batches;
    const int64_t tile_cols = (int64_t)tile_batches * kBatch;
    const int64_t ncols = t == ntile - 1 ? ncols_last : tile_cols;
    const T* base = Phi + (int64_t)roff[t] * tile_cols;   // every tile before t is full
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t c0 = (int64_t)(b - t * tile_batches) * kBatch;
    double sw[4];
    for (int u = 0; u < 4; ++u) sw[u] = sqrt(pw[(int64_t)b * kBatch + lane + 64 * u]);
    const int nB = roff[t + 1] - roff[t];
    for (int k = wave; k < nB; k += 4) {
        const T* row = base + (int64_t)k * ncols + c0;
        double v = 0.0;
        for (int u = 0; u < 4; ++u) v = fmax(v, sw[u] * fabs((double)row[lane + 64 * u]));
        for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
        if (lane == 0) out[(int64_t)b * ld + k] = v;
    }
}

// One workgroup per batch: fs[b][A] = max over the functions mu of shell A of Ft[b][mu].
__global__ __launch_bounds__(256) void shellmax_kernel(const double* __restrict__ Ft, int64_t ldf,
                                                       const int32_t* __restrict__ shell_l,
                                                       const int32_t* __restrict__ shell_row, int32_t nshell,
                                                       double* __restrict__ fs)
{
    const int b = blockIdx.x;
    const double* f = Ft + (int64_t)b * ldf;
    for (int A = threadIdx.x; A < nshell; A += blockDim.x) {
        const int r = shell_row[A], n = (shell_l[A] + 1) * (shell_l[A] + 2) / 2;
        double m = 0.0;
        for (int k = 0; k < n; ++k) m = fmax(m, f[r + k]);
        fs[(int64_t)b * nshell + A] = m;
    }
}

hipError_t launch_phimax(const double* Phi, const float* Phi32, const int32_t* roff, int32_t ntile,
                         int32_t tile_batches, int64_t ncols_last, const double* pw, int32_t nbatch, double* out,
                         int64_t ld, hipStream_t s)
{
    if (nbatch <= 0) return hipSuccess;
    if ((!Phi && !Phi32) || !roff || !pw || !out || tile_batches < 1 || ntile < 1 ||
        (int64_t)ntile * tile_batches < nbatch)
        return hipErrorInvalidValue;
    if (Phi32)
        hipLaunchKernelGGL((phimax_kernel<float>), dim3(nbatch), dim3(kBatch), 0, s, Phi32, roff, ntile, tile_batches,
                           ncols_last, pw, out, ld);
    else
        hipLaunchKernelGGL((phimax_kernel<double>), dim3(nbatch), dim3(kBatch), 0, s, Phi, roff, ntile, tile_batches,
                           ncols_last, pw, out, ld);
    return hipGetLastError();
}

hipError_t launch_shellmax(const double* Ft, int64_t ldf, const int32_t* shell_l, const int32_t* shell_row,
                           int32_t nshell, int32_t nbatch, double* fs, hipStream_t s)
{
    if (nbatch <= 0 || nshell <= 0) return hipSuccess;
    hipLaunchKernelGGL(shellmax_kernel, dim3(nbatch), dim3(256), 0, s, Ft, ldf, shell_l, shell_row, nshell, fs);
    return hipGetLastError();
}

hipError_t launch_phisum(const double* Phi, const float* Phi32, const int32_t* roff, int32_t ntile,
                         int32_t tile_batches, int64_t ncols_last, const double* pw, int32_t nbatch, double* phit,
                         hipStream_t s)
{
    if (nbatch <= 0) return hipSuccess;
    if ((!Phi && !Phi32) || !roff || !pw || !phit || tile_batches < 1 || ntile < 1 ||
        (int64_t)ntile * tile_batches < nbatch)
        return hipErrorInvalidValue;
    if (Phi32)
        hipLaunchKernelGGL((phisum_kernel<float>), dim3(nbatch), dim3(kBatch), 0, s, Phi32, roff, ntile, tile_batches,
                           ncols_last, pw, phit);
    else
        hipLaunchKernelGGL((phisum_kernel<double>), dim3(nbatch), dim3(kBatch), 0, s, Phi, roff, ntile, tile_batches,
                           ncols_last, pw, phit);
    return hipGetLastError();
}

hipError_t launch_screen_est(const EstArgs& a, hipStream_t s)
{
    if (a.nbatch <= 0) return hipSuccess;
    const size_t shm = (size_t)2 * a.nshell * sizeof(int32_t);
    hipLaunchKernelGGL(screen_est_kernel, dim3(a.nbatch), dim3(256), shm, s, a);
    return hipGetLastError();
}

hipError_t launch_screen_scan(const int32_t* counts, int32_t nbatch, int32_t nlist, int64_t* run_base,
                              int64_t* bt_base, hipStream_t s)
{
    hipLaunchKernelGGL(screen_scan_kernel, dim3(nlist), dim3(256), 0, s, counts, nbatch, nlist, run_base, bt_base);
    return hipGetLastError();
}

}  // namespace snk
