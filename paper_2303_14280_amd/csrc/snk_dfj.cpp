// Host runtime of the density-fitted Coulomb matrix (Sec. II.B): primitive-pair and
// auxiliary-shell tables, the metric and its Cholesky factor at set-up, and the build
// sequence of Eqs. Dp, V_df / cabP-jengine, P_df and J_df on one stream.
#include "snk.h"
#include "snk_dfj.h"
#include "snk_internal.h"

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

using namespace snk;

namespace snk {
void set_last_error(const char* msg);   // error text of context-free calls (snk_host.cpp)
}

struct snk_dfj {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t nbf = 0, nauxf = 0;
    int32_t naux = 0;                      // auxiliary shells
    int32_t npp = 0, nsp = 0;
    int32_t cls_beg[7] = {};               // primitive pairs of class c: cls_beg[c] .. cls_beg[c + 1]
    int32_t lbeg[4] = {};                  // auxiliary shells of l: lbeg[l] .. lbeg[l + 1] (sorted by l)
    int32_t lp_slot[6] = {};               // first slot of the chunks of primitive-pair total LP
    int32_t nslot = 0;
    DfjPrim* d_pp = nullptr;
    DfjShellPair* d_sp = nullptr;
    DfjAux* d_aux = nullptr;
    int32_t* d_lbeg = nullptr;
    double* d_tab = nullptr;
    double* d_Dh = nullptr;                // [npp][kDfjHerm]
    double* d_Jpp = nullptr;               // [npp][kDfjCart]
    double* d_jh = nullptr;                // Hermite J partial sums of one class's launch, per auxiliary chunk
    double* d_part = nullptr;              // [naux][nslot][kDfjAuxHerm]
    double* d_Dc = nullptr;                // [naux][kDfjAuxHerm]
    double* d_L = nullptr;                 // [nauxf][nauxf] L^-1 of the Cholesky factor L (lower)
    double* d_U = nullptr;                 // its transpose L^-T
    double* d_v = nullptr;
    double* d_y = nullptr;
    double* d_d = nullptr;
    double* d_P = nullptr;                 // host-pointer mode staging
    double* d_J = nullptr;
    double* d_ej = nullptr;
    int32_t* d_status = nullptr;
    std::string err;
};

namespace {

constexpr int kVauxChunk = 2048;          // orbital primitive pairs per workgroup of the v step
constexpr double kPairCut = 1e-24;        // |exp(-mu AB^2) c_a c_b| below which a primitive pair is dropped

int dfj_err(snk_dfj* c, const std::string& m, int code)
{
    if (c) c->err = m;
    set_last_error(m.c_str());
    return code;
}

#define DFJ_HIP(c, expr)                                                                               \
    do {                                                                                               \
        const hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                          \
            return dfj_err(c, std::string(#expr) + ": " + hipGetErrorString(e_),                       \
                           e_ == hipErrorOutOfMemory ? SNK_E_NOMEM : SNK_E_DEVICE);                    \
    } while (0)

template <typename T>
int dfj_alloc(snk_dfj* c, T** p, size_t n)
{
    DFJ_HIP(c, hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T)));
    return SNK_OK;
}

template <typename T>
int dfj_upload(snk_dfj* c, T** p, const std::vector<T>& v)
{
    int rc = dfj_alloc(c, p, v.size());
    if (rc) return rc;
    if (!v.empty()) DFJ_HIP(c, hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return SNK_OK;
}

int check_basis(snk_dfj* c, const snk_basis* b, const char* what, bool one_prim)
{
    const std::string w(what);
    if (!b || b->nshell < 1 || !b->center || !b->l || !b->nprim || !b->prim_off || !b->exps || !b->coefs)
        return dfj_err(c, w + ": NULL or empty basis", SNK_E_ARG);
    for (int s = 0; s < b->nshell; ++s) {
        if (b->l[s] < 0 || b->l[s] > SNK_MAX_L) return dfj_err(c, w + ": angular momentum outside 0..2", SNK_E_ARG);
        if (b->nprim[s] < 1 || b->nprim[s] > SNK_MAX_NPRIM || (one_prim && b->nprim[s] != 1))
            return dfj_err(c, w + (one_prim ? ": auxiliary shells take one primitive" : ": primitive count outside 1..8"),
                           SNK_E_ARG);
        if (b->prim_off[s] < 0) return dfj_err(c, w + ": negative primitive offset", SNK_E_ARG);
        for (int d = 0; d < 3; ++d)
            if (!std::isfinite(b->center[3 * s + d])) return dfj_err(c, w + ": non-finite centre", SNK_E_ARG);
        for (int k = 0; k < b->nprim[s]; ++k) {
            const double e = b->exps[b->prim_off[s] + k], cf = b->coefs[b->prim_off[s] + k];
            if (!std::isfinite(e) || !(e > 0.0) || !std::isfinite(cf))
                return dfj_err(c, w + ": exponent not finite and positive, or non-finite coefficient", SNK_E_ARG);
        }
    }
    return SNK_OK;
}

int ncart_h(int l) { return (l + 1) * (l + 2) / 2; }

int class_of(int la, int lb) { return la == 0 ? 0 : (la == 1 ? (lb == 0 ? 1 : 2) : 3 + lb); }
constexpr int kClassLP[6] = {0, 1, 2, 2, 3, 4};
constexpr int kClassLA[6] = {0, 1, 1, 2, 2, 2};
constexpr int kClassLB[6] = {0, 0, 1, 0, 1, 2};

void free_dfj(snk_dfj* c)
{
    if (!c) return;
    for (void* p : {(void*)c->d_pp, (void*)c->d_sp, (void*)c->d_aux, (void*)c->d_lbeg, (void*)c->d_tab,
                    (void*)c->d_Dh, (void*)c->d_Jpp, (void*)c->d_jh, (void*)c->d_part, (void*)c->d_Dc, (void*)c->d_L, (void*)c->d_U,
                    (void*)c->d_v, (void*)c->d_y, (void*)c->d_d, (void*)c->d_P, (void*)c->d_J, (void*)c->d_ej,
                    (void*)c->d_status})
        (void)hipFree(p);
    delete c;
}

int setup(snk_dfj* c, const snk_basis* b, const snk_basis* a)
{
    // function offsets
    std::vector<int32_t> fo(b->nshell + 1, 0), fa(a->nshell + 1, 0);
    for (int s = 0; s < b->nshell; ++s) fo[s + 1] = fo[s] + ncart_h(b->l[s]);
    for (int s = 0; s < a->nshell; ++s) fa[s + 1] = fa[s] + ncart_h(a->l[s]);
    c->nbf = fo[b->nshell];
    c->nauxf = fa[a->nshell];
    c->naux = a->nshell;

    // orbital shell pairs by class, their primitive pairs consecutive
    std::vector<std::vector<DfjShellPair>> sp(6);
    std::vector<std::vector<DfjPrim>> pp(6);
    for (int s = 0; s < b->nshell; ++s)
        for (int t = 0; t <= s; ++t) {
            int A = s, B = t;
            if (b->l[B] > b->l[A]) std::swap(A, B);
            const int cls = class_of(b->l[A], b->l[B]);
            const double* RA = b->center + 3 * A;
            const double* RB = b->center + 3 * B;
            const double AB[3] = {RA[0] - RB[0], RA[1] - RB[1], RA[2] - RB[2]};
            const double ab2 = AB[0] * AB[0] + AB[1] * AB[1] + AB[2] * AB[2];
            DfjShellPair h{fo[A], fo[B], b->l[A], b->l[B], (int32_t)pp[cls].size(), 0};
            for (int i = 0; i < b->nprim[A]; ++i)
                for (int j = 0; j < b->nprim[B]; ++j) {
                    const double za = b->exps[b->prim_off[A] + i], zb = b->exps[b->prim_off[B] + j];
                    const double ca = b->coefs[b->prim_off[A] + i], cb = b->coefs[b->prim_off[B] + j];
                    const double zp = za + zb;
                    if (std::fabs(std::exp(-za * zb / zp * ab2) * ca * cb) < kPairCut) continue;
                    DfjPrim q{};
                    q.Px = (za * RA[0] + zb * RB[0]) / zp;
                    q.Py = (za * RA[1] + zb * RB[1]) / zp;
                    q.Pz = (za * RA[2] + zb * RB[2]) / zp;
                    q.za = za;
                    q.zb = zb;
                    q.ABx = AB[0];
                    q.ABy = AB[1];
                    q.ABz = AB[2];
                    q.cc1 = ca * cb;
                    q.cc = (A == B ? 1.0 : 2.0) * ca * cb;
                    q.fa = fo[A];
                    q.fb = fo[B];
                    pp[cls].push_back(q);
                }
            h.np = (int32_t)pp[cls].size() - h.pbeg;
            sp[cls].push_back(h);
        }
    std::vector<DfjPrim> allpp;
    std::vector<DfjShellPair> allsp;
    for (int cls = 0; cls < 6; ++cls) {
        c->cls_beg[cls] = (int32_t)allpp.size();
        for (DfjShellPair h : sp[cls]) {
            h.pbeg += c->cls_beg[cls];
            allsp.push_back(h);
        }
        allpp.insert(allpp.end(), pp[cls].begin(), pp[cls].end());
    }
    c->cls_beg[6] = (int32_t)allpp.size();
    c->npp = (int32_t)allpp.size();
    c->nsp = (int32_t)allsp.size();

    // auxiliary shells sorted by l, each keeping its function offset in the caller's order
    std::vector<DfjAux> aux;
    for (int l = 0; l <= 2; ++l) {
        c->lbeg[l] = (int32_t)aux.size();
        for (int s = 0; s < a->nshell; ++s) {
            if (a->l[s] != l) continue;
            const double* R = a->center + 3 * s;
            aux.push_back(DfjAux{R[0], R[1], R[2], a->exps[a->prim_off[s]], a->coefs[a->prim_off[s]], l, fa[s]});
        }
    }
    c->lbeg[3] = (int32_t)aux.size();

    // slots of the v step: chunks of the primitive pairs of each total LP (classes with the
    // same LP are adjacent)
    c->nslot = 0;
    for (int lp = 0; lp <= 4; ++lp) {
        c->lp_slot[lp] = c->nslot;
        int32_t b0 = -1, b1 = -1;
        for (int cls = 0; cls < 6; ++cls)
            if (kClassLP[cls] == lp) {
                if (b0 < 0) b0 = c->cls_beg[cls];
                b1 = c->cls_beg[cls + 1];
            }
        if (b1 > b0) c->nslot += (b1 - b0 + kVauxChunk - 1) / kVauxChunk;
    }
    c->lp_slot[5] = c->nslot;

    int rc;
    // the J digestion's workspace: the largest class launch
    size_t jh = 1;
    for (int cls = 0; cls < 6; ++cls) {
        const int32_t n = c->cls_beg[cls + 1] - c->cls_beg[cls];
        const int lp = kClassLP[cls];
        if (n > 0)
            jh = std::max(jh, (size_t)dfj_jpair_chunks(n, c->naux) * n * ((lp + 1) * (lp + 2) * (lp + 3) / 6));
    }
    if ((rc = dfj_alloc(c, &c->d_jh, jh))) return rc;
    const std::vector<double> tab = boys_table_cols(kDfjBoysCols);
    const std::vector<int32_t> lb(c->lbeg, c->lbeg + 4);
    if ((rc = dfj_upload(c, &c->d_pp, allpp)) || (rc = dfj_upload(c, &c->d_sp, allsp)) ||
        (rc = dfj_upload(c, &c->d_aux, aux)) || (rc = dfj_upload(c, &c->d_lbeg, lb)) ||
        (rc = dfj_upload(c, &c->d_tab, tab)) || (rc = dfj_alloc(c, &c->d_Dh, (size_t)c->npp * kDfjHerm)) ||
        (rc = dfj_alloc(c, &c->d_Jpp, (size_t)c->npp * kDfjCart)) ||
        (rc = dfj_alloc(c, &c->d_part, (size_t)c->naux * std::max(1, c->nslot) * kDfjAuxHerm)) ||
        (rc = dfj_alloc(c, &c->d_Dc, (size_t)c->naux * kDfjAuxHerm)) ||
        (rc = dfj_alloc(c, &c->d_L, (size_t)c->nauxf * c->nauxf)) ||
        (rc = dfj_alloc(c, &c->d_U, (size_t)c->nauxf * c->nauxf)) || (rc = dfj_alloc(c, &c->d_v, c->nauxf)) ||
        (rc = dfj_alloc(c, &c->d_y, c->nauxf)) || (rc = dfj_alloc(c, &c->d_d, c->nauxf)) ||
        (rc = dfj_alloc(c, &c->d_P, (size_t)c->nbf * c->nbf)) || (rc = dfj_alloc(c, &c->d_J, (size_t)c->nbf * c->nbf)) ||
        (rc = dfj_alloc(c, &c->d_ej, 1)) || (rc = dfj_alloc(c, &c->d_status, 1)))
        return rc;
    // the metric and its factor (Eq. P_df's V, once per auxiliary basis)
    DFJ_HIP(c, hipMemsetAsync(c->d_status, 0, sizeof(int32_t), c->stream));
    DFJ_HIP(c, launch_dfj_metric(c->d_aux, c->naux, c->d_tab, c->d_L, c->nauxf, c->stream));
    DFJ_HIP(c, launch_dfj_cholesky(c->d_L, c->nauxf, c->d_status, c->stream));
    int32_t status = 0;
    DFJ_HIP(c, hipMemcpyAsync(&status, c->d_status, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    DFJ_HIP(c, hipStreamSynchronize(c->stream));
    if (status) return dfj_err(c, "auxiliary metric not positive definite (linearly dependent functions)", SNK_E_ARG);
    // V^-1 = L^-T L^-1: the inverse factor once, so that a build's solve is two triangular
    // products
    DFJ_HIP(c, launch_dfj_invert(c->d_L, c->nauxf, c->d_U, c->stream));
    DFJ_HIP(c, hipStreamSynchronize(c->stream));
    return SNK_OK;
}

}  // namespace

extern "C" {

int snk_dfj_create(const snk_basis* basis, const snk_basis* aux, int device, void* stream, snk_dfj** out)
{
    if (!out) return dfj_err(nullptr, "output context pointer is NULL", SNK_E_ARG);
    *out = nullptr;
    int rc = check_basis(nullptr, basis, "orbital basis", false);
    if (rc) return rc;
    if ((rc = check_basis(nullptr, aux, "auxiliary basis", true))) return rc;
    snk_dfj* c = new (std::nothrow) snk_dfj();
    if (!c) return SNK_E_NOMEM;
    c->device = device;
    c->stream = (hipStream_t)stream;
    const hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) {
        dfj_err(c, std::string("hipSetDevice: ") + hipGetErrorString(e), SNK_E_DEVICE);
        free_dfj(c);
        return SNK_E_DEVICE;
    }
    if ((rc = setup(c, basis, aux))) {
        set_last_error(c->err.c_str());
        free_dfj(c);
        return rc;
    }
    *out = c;
    return SNK_OK;
}

int snk_dfj_build(snk_dfj* c, const double* P, double* J_out, double* v_out, double* d_out, double* ej_out,
                  uint32_t flags)
{
    if (!c) return dfj_err(nullptr, "context is NULL", SNK_E_ARG);
    if (!P || !J_out) return dfj_err(c, "P or J_out is NULL", SNK_E_ARG);
    if (flags & ~(uint32_t)SNK_DEVICE_PTRS) return dfj_err(c, "unknown flag", SNK_E_ARG);
    const bool dev = (flags & SNK_DEVICE_PTRS) != 0;
    DFJ_HIP(c, hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const int64_t nbf = c->nbf, nb2 = nbf * nbf;
    const double* dP = P;
    double* dJ = dev ? J_out : c->d_J;
    if (!dev) {
        DFJ_HIP(c, hipMemcpyAsync(c->d_P, P, nb2 * sizeof(double), hipMemcpyHostToDevice, s));
        dP = c->d_P;
    }
    // Eq. Dp per class
    for (int cls = 0; cls < 6; ++cls)
        DFJ_HIP(c, launch_dfj_hdens(cls, c->d_pp + c->cls_beg[cls], c->cls_beg[cls + 1] - c->cls_beg[cls], dP, nbf,
                                    c->d_Dh + (int64_t)c->cls_beg[cls] * kDfjHerm, s));
    // Eqs. V_df / cabP-jengine: every (LP, LC) class pair
    for (int lp = 0; lp <= 4; ++lp) {
        int32_t b0 = -1, b1 = -1;
        for (int cls = 0; cls < 6; ++cls)
            if (kClassLP[cls] == lp) {
                if (b0 < 0) b0 = c->cls_beg[cls];
                b1 = c->cls_beg[cls + 1];
            }
        if (b1 <= b0) continue;
        for (int lc = 0; lc <= 2; ++lc)
            DFJ_HIP(c, launch_dfj_vaux(lp, lc, c->d_pp, c->d_Dh, b0, b1, kVauxChunk, c->lp_slot[lp], c->d_aux,
                                       c->lbeg[lc], c->lbeg[lc + 1], c->nslot, c->d_tab, c->d_part, s));
    }
    double* dv = (dev && v_out) ? v_out : c->d_v;
    double* dd = (dev && d_out) ? d_out : c->d_d;
    DFJ_HIP(c, launch_dfj_vfinish(c->d_aux, c->naux, c->d_part, c->nslot, dv, s));
    // Eq. P_df
    DFJ_HIP(c, launch_dfj_solve(c->d_L, c->d_U, c->nauxf, dv, c->d_y, dd, s));
    // Eq. J_df
    DFJ_HIP(c, launch_dfj_auxdens(c->d_aux, c->naux, dd, c->d_Dc, s));
    for (int cls = 0; cls < 6; ++cls)
        DFJ_HIP(c, launch_dfj_jpair(cls, c->d_pp + c->cls_beg[cls], c->cls_beg[cls + 1] - c->cls_beg[cls], c->d_aux,
                                    c->naux, c->d_Dc, c->d_lbeg, c->d_tab, c->d_jh,
                                    c->d_Jpp + (int64_t)c->cls_beg[cls] * kDfjCart, s));
    DFJ_HIP(c, launch_dfj_jcollect(c->d_sp, c->nsp, c->d_Jpp, dJ, nbf, s));
    if (ej_out) DFJ_HIP(c, launch_dfj_dot(dP, dJ, nb2, c->d_ej, s));
    if (!dev) {
        DFJ_HIP(c, hipMemcpyAsync(J_out, dJ, nb2 * sizeof(double), hipMemcpyDeviceToHost, s));
        if (v_out) DFJ_HIP(c, hipMemcpyAsync(v_out, dv, c->nauxf * sizeof(double), hipMemcpyDeviceToHost, s));
        if (d_out) DFJ_HIP(c, hipMemcpyAsync(d_out, dd, c->nauxf * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    if (ej_out) {
        double ej = 0.0;
        DFJ_HIP(c, hipMemcpyAsync(&ej, c->d_ej, sizeof(double), hipMemcpyDeviceToHost, s));
        DFJ_HIP(c, hipStreamSynchronize(s));
        *ej_out = 0.5 * ej;
    } else if (!dev) {
        DFJ_HIP(c, hipStreamSynchronize(s));
    }
    return SNK_OK;
}

int64_t snk_dfj_naux(const snk_dfj* c) { return c ? c->nauxf : 0; }

const char* snk_dfj_last_error(const snk_dfj* c) { return c ? c->err.c_str() : ""; }

void snk_dfj_destroy(snk_dfj* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    free_dfj(c);
}

}  // extern "C"
