// C ABI entry points: grid and model objects, argument checks, dispatch to
// the HIP kernels, error reporting.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "cm_impl.hpp"

namespace cm {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

cm_status hip_fail(hipError_t e, const char* where)
{
    set_error(std::string(where) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? CM_ERR_ALLOC : CM_ERR_HIP;
}

// GLL nodes and weights for N = 4 in closed form; differentiation matrix from
// barycentric weights, D_ij = (lambda_j / lambda_i) / (x_i - x_j), with the
// diagonal set to minus the off-diagonal row sum (so D annihilates constants).
static void gll4(double* xi, double* w, double* D)
{
    const double a = std::sqrt(3.0 / 7.0);
    const double x[NQ] = {-1.0, -a, 0.0, a, 1.0};
    const double ww[NQ] = {1.0 / 10.0, 49.0 / 90.0, 32.0 / 45.0, 49.0 / 90.0, 1.0 / 10.0};
    double lam[NQ];
    for (int j = 0; j < NQ; ++j) {
        double p = 1.0;
        for (int k = 0; k < NQ; ++k)
            if (k != j) p *= (x[j] - x[k]);
        lam[j] = 1.0 / p;
    }
    for (int i = 0; i < NQ; ++i) {
        xi[i] = x[i];
        w[i] = ww[i];
        double s = 0.0;
        for (int j = 0; j < NQ; ++j) {
            if (j == i) continue;
            double d = (lam[j] / lam[i]) / (x[i] - x[j]);
            D[i * NQ + j] = d;
            s += d;
        }
        D[i * NQ + i] = -s;
    }
}

static inline int64_t node_index(const cm_grid* g, int ex, int ey, int ez, int i, int j, int k)
{
    int64_t e = ex + (int64_t)g->desc.ne[0] * (ey + (int64_t)g->desc.ne[1] * ez);
    return e * NP + i + NQ * (j + NQ * k);
}

// coordinates and (cross-product form) metric terms on the host, FP64
static void build_geometry(cm_grid* g)
{
    const cm_grid_desc& d = g->desc;
    const int64_t nn = g->n_nodes;
    g->xyz.assign(3 * nn, 0.0);
    const double ztop = d.hi[2], zlo = d.lo[2];
    for (int ez = 0; ez < d.ne[2]; ++ez)
        for (int ey = 0; ey < d.ne[1]; ++ey)
            for (int ex = 0; ex < d.ne[0]; ++ex)
                for (int k = 0; k < NQ; ++k)
                    for (int j = 0; j < NQ; ++j)
                        for (int i = 0; i < NQ; ++i) {
                            int64_t n = node_index(g, ex, ey, ez, i, j, k);
                            double x = d.lo[0] + (ex + 0.5 * (1.0 + g->xi[i])) * g->h[0];
                            double y = d.lo[1] + (ey + 0.5 * (1.0 + g->xi[j])) * g->h[1];
                            double z = d.lo[2] + (ez + 0.5 * (1.0 + g->xi[k])) * g->h[2];
                            if (d.topo == 1) {
                                double r = x - d.topo_xc;
                                double zs = d.topo_h * d.topo_a * d.topo_a / (r * r + d.topo_a * d.topo_a);
                                z += zs * (ztop - z) / (ztop - zlo);
                            }
                            g->xyz[n] = x;
                            g->xyz[nn + n] = y;
                            g->xyz[2 * nn + n] = z;
                        }
    g->Ja.assign(9 * nn, 0.0);
    g->J.assign(nn, 0.0);
    if (d.topo == 0) {
        const double hx = g->h[0], hy = g->h[1], hz = g->h[2];
        for (int64_t n = 0; n < nn; ++n) {
            g->Ja[0 * nn + n] = 0.25 * hy * hz;
            g->Ja[4 * nn + n] = 0.25 * hx * hz;
            g->Ja[8 * nn + n] = 0.25 * hx * hy;
            g->J[n] = 0.125 * hx * hy * hz;
        }
        return;
    }
    // warped: dX[d][c] = sum_l D_{.,l} x_c along reference direction d
    for (int64_t e = 0; e < g->n_elem; ++e)
        for (int k = 0; k < NQ; ++k)
            for (int j = 0; j < NQ; ++j)
                for (int i = 0; i < NQ; ++i) {
                    int64_t n = e * NP + i + NQ * (j + NQ * k);
                    double dX[3][3];
                    for (int c = 0; c < 3; ++c) {
                        const double* f = g->xyz.data() + c * nn + e * NP;
                        double s0 = 0, s1 = 0, s2 = 0;
                        for (int l = 0; l < NQ; ++l) {
                            s0 += g->D[i * NQ + l] * f[l + NQ * (j + NQ * k)];
                            s1 += g->D[j * NQ + l] * f[i + NQ * (l + NQ * k)];
                            s2 += g->D[k * NQ + l] * f[i + NQ * (j + NQ * l)];
                        }
                        dX[0][c] = s0;
                        dX[1][c] = s1;
                        dX[2][c] = s2;
                    }
                    for (int dd = 0; dd < 3; ++dd) {
                        const double* a = dX[(dd + 1) % 3];
                        const double* b = dX[(dd + 2) % 3];
                        g->Ja[(3 * dd + 0) * nn + n] = a[1] * b[2] - a[2] * b[1];
                        g->Ja[(3 * dd + 1) * nn + n] = a[2] * b[0] - a[0] * b[2];
                        g->Ja[(3 * dd + 2) * nn + n] = a[0] * b[1] - a[1] * b[0];
                    }
                    g->J[n] = dX[0][0] * g->Ja[0 * nn + n] + dX[0][1] * g->Ja[1 * nn + n] +
                              dX[0][2] * g->Ja[2 * nn + n];
                }
}

cm_model::ProfRec* prof_begin(cm_model* m, int kind, hipStream_t s)
{
    if (!m->profiling) return nullptr;
    if (m->prof_used == m->prof.size()) {
        cm_model::ProfRec r;
        if (hipEventCreate(&r.a) != hipSuccess) return nullptr;
        if (hipEventCreate(&r.b) != hipSuccess) { (void)hipEventDestroy(r.a); return nullptr; }
        m->prof.push_back(r);
    }
    cm_model::ProfRec* r = &m->prof[m->prof_used++];
    r->kind = kind;
    (void)hipEventRecord(r->a, s);
    return r;
}

void prof_end(cm_model::ProfRec* r, hipStream_t s)
{
    if (r) (void)hipEventRecord(r->b, s);
}

}  // namespace cm

using namespace cm;

#define CM_TRY_HIP(expr, where)                      \
    do {                                             \
        hipError_t _e = (expr);                      \
        if (_e != hipSuccess) return hip_fail(_e, where); \
    } while (0)

// Traversal table of the elements.  Blocks are dealt round-robin to the
// eight XCDs, so XCD x works on the contiguous index range
// [x q + min(x, r), +q + (x < r)) of n = 8 q + r elements; inside that range
// the elements are visited in column tiles of TX x TY elements in (x, y)
// over all layers of the range, so that most face neighbours of the
// elements in flight on an XCD are in flight there too (shared L2).
static void element_order(const cm_grid_desc& d, std::vector<int>& ord)
{
#ifndef CM_ORDER_TX
#define CM_ORDER_TX 8
#define CM_ORDER_TY 4
#endif
    constexpr int TX = CM_ORDER_TX, TY = CM_ORDER_TY;
    const int64_t ne0 = d.ne[0], ne1 = d.ne[1], ne2 = d.ne[2];
    const int64_t n = ne0 * ne1 * ne2, q = n / 8, r = n % 8;
    const int64_t ntx = (ne0 + TX - 1) / TX;
    ord.resize(n);
    std::vector<std::pair<int64_t, int>> keyed;
    for (int64_t x = 0; x < 8; ++x) {
        const int64_t g0 = x * q + std::min(x, r), gs = q + (x < r ? 1 : 0);
        keyed.resize(gs);
        for (int64_t s = 0; s < gs; ++s) {
            const int64_t e = g0 + s;
            const int64_t ex = e % ne0, ey = (e / ne0) % ne1, ez = e / (ne0 * ne1);
#ifdef CM_ORDER_LINEAR
            const int64_t key = e;
#else
            const int64_t key = (((ey / TY * ntx + ex / TX) * ne2 + ez) * TY + ey % TY) * TX + ex % TX;
#endif
            keyed[s] = {key, (int)e};
        }
        std::sort(keyed.begin(), keyed.end());
        for (int64_t s = 0; s < gs; ++s) ord[g0 + s] = keyed[s].second;
    }
}

extern "C" {

const char* cm_last_error(void) { return g_err.c_str(); }

cm_status cm_grid_create(const cm_grid_desc* desc, int hip_device, cm_grid** out)
{
    if (!desc || !out) { set_error("cm_grid_create: null argument"); return CM_ERR_ARG; }
    *out = nullptr;
    if (desc->N != 4) { set_error("cm_grid_create: only N = 4 is supported"); return CM_ERR_UNSUPPORTED; }
    for (int a = 0; a < 3; ++a) {
        if (desc->ne[a] < 1 || !(desc->hi[a] > desc->lo[a])) {
            set_error("cm_grid_create: need ne >= 1 and hi > lo in every direction");
            return CM_ERR_ARG;
        }
    }
    if (desc->topo != 0 && desc->topo != 1) { set_error("cm_grid_create: topo must be 0 or 1"); return CM_ERR_ARG; }
    if (desc->topo == 1 && !(desc->topo_a > 0.0)) { set_error("cm_grid_create: topo_a must be > 0"); return CM_ERR_ARG; }
    int64_t ne = (int64_t)desc->ne[0] * desc->ne[1] * desc->ne[2];
    if (ne * NP * 16 >= ((int64_t)1 << 31)) { set_error("cm_grid_create: grid too large for 32-bit kernel indexing"); return CM_ERR_UNSUPPORTED; }
    int ndev = 0;
    CM_TRY_HIP(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
    if (hip_device < 0 || hip_device >= ndev) { set_error("cm_grid_create: bad device ordinal"); return CM_ERR_ARG; }
    cm_grid* g = new (std::nothrow) cm_grid();
    if (!g) { set_error("cm_grid_create: out of host memory"); return CM_ERR_ALLOC; }
    g->device = hip_device;
    g->desc = *desc;
    g->n_elem = ne;
    g->n_nodes = ne * NP;
    for (int a = 0; a < 3; ++a) g->h[a] = (desc->hi[a] - desc->lo[a]) / desc->ne[a];
    gll4(g->xi, g->w, g->D);
    double hmin = std::fmin(g->h[0], std::fmin(g->h[1], g->h[2]));
    g->dmin = hmin * 0.5 * (g->xi[1] - g->xi[0]);
    try {
        build_geometry(g);
    } catch (const std::bad_alloc&) {
        delete g;
        set_error("cm_grid_create: out of host memory");
        return CM_ERR_ALLOC;
    }
    hipError_t e = hipSetDevice(hip_device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&g->n_cu, hipDeviceAttributeMultiprocessorCount, hip_device);
    if (e == hipSuccess) {
        std::vector<int> ord;
        element_order(*desc, ord);
        e = hipMalloc(&g->d_order, sizeof(int) * ord.size());
        if (e == hipSuccess) e = hipMemcpy(g->d_order, ord.data(), sizeof(int) * ord.size(), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && desc->topo == 1) {
        const int64_t nn = g->n_nodes;
        std::vector<double> m64(10 * nn);
        std::vector<float> m32(10 * nn);
        for (int q = 0; q < 9; ++q)
            for (int64_t n = 0; n < nn; ++n) m64[q * nn + n] = g->Ja[q * nn + n];
        for (int64_t n = 0; n < nn; ++n) m64[9 * nn + n] = 1.0 / g->J[n];
        for (int64_t q = 0; q < 10 * nn; ++q) m32[q] = (float)m64[q];
        e = hipMalloc(&g->d_metrics64, sizeof(double) * 10 * nn);
        if (e == hipSuccess) e = hipMalloc(&g->d_metrics32, sizeof(float) * 10 * nn);
        if (e == hipSuccess) e = hipMalloc(&g->d_z, sizeof(double) * nn);
        if (e == hipSuccess) e = hipMemcpy(g->d_metrics64, m64.data(), sizeof(double) * 10 * nn, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(g->d_metrics32, m32.data(), sizeof(float) * 10 * nn, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(g->d_z, g->xyz.data() + 2 * nn, sizeof(double) * nn, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = upload_constants(g);
    if (e != hipSuccess) {
        cm_status st = hip_fail(e, "cm_grid_create");
        cm_grid_destroy(g);
        return st;
    }
    *out = g;
    return CM_OK;
}

cm_status cm_grid_destroy(cm_grid* g)
{
    if (!g) return CM_OK;
    (void)hipSetDevice(g->device);
    if (g->d_metrics64) (void)hipFree(g->d_metrics64);
    if (g->d_metrics32) (void)hipFree(g->d_metrics32);
    if (g->d_z) (void)hipFree(g->d_z);
    if (g->d_order) (void)hipFree(g->d_order);
    delete g;
    return CM_OK;
}

cm_status cm_grid_query(const cm_grid* g, cm_grid_info* out)
{
    if (!g || !out) { set_error("cm_grid_query: null argument"); return CM_ERR_ARG; }
    out->n_elem = g->n_elem;
    out->n_nodes = g->n_nodes;
    out->state_stride = g->n_elem * SRUN;
    out->N = 4;
    out->warped = g->desc.topo;
    out->dmin_node = g->dmin;
    return CM_OK;
}

cm_status cm_grid_copy_coords(const cm_grid* g, double* xyz)
{
    if (!g || !xyz) { set_error("cm_grid_copy_coords: null argument"); return CM_ERR_ARG; }
    std::memcpy(xyz, g->xyz.data(), sizeof(double) * 3 * g->n_nodes);
    return CM_OK;
}

cm_status cm_grid_copy_wJ(const cm_grid* g, double* wJ)
{
    if (!g || !wJ) { set_error("cm_grid_copy_wJ: null argument"); return CM_ERR_ARG; }
    for (int64_t e = 0; e < g->n_elem; ++e)
        for (int k = 0; k < NQ; ++k)
            for (int j = 0; j < NQ; ++j)
                for (int i = 0; i < NQ; ++i) {
                    int64_t n = e * NP + i + NQ * (j + NQ * k);
                    wJ[n] = g->w[i] * g->w[j] * g->w[k] * g->J[n];
                }
    return CM_OK;
}

cm_status cm_grid_copy_metrics(const cm_grid* g, double* Ja, double* J)
{
    if (!g || !Ja || !J) { set_error("cm_grid_copy_metrics: null argument"); return CM_ERR_ARG; }
    std::memcpy(Ja, g->Ja.data(), sizeof(double) * 9 * g->n_nodes);
    std::memcpy(J, g->J.data(), sizeof(double) * g->n_nodes);
    return CM_OK;
}

cm_status cm_model_destroy(cm_model* m)
{
    if (!m) return CM_OK;
    (void)hipSetDevice(m->device);
    if (m->d_F2) (void)hipFree(m->d_F2);
    for (int q = 0; q < 2; ++q)
        if (m->d_T[q]) (void)hipFree(m->d_T[q]);
    if (m->d_pr) (void)hipFree(m->d_pr);
    if (m->d_rhor) (void)hipFree(m->d_rhor);
    if (m->d_Yref) (void)hipFree(m->d_Yref);
    if (m->d_bg32) (void)hipFree(m->d_bg32);
    if (m->d_bg64) (void)hipFree(m->d_bg64);
    if (m->d_partials) (void)hipFree(m->d_partials);
    if (m->d_mlp_w) (void)hipFree(m->d_mlp_w);
    if (m->d_mlp_norm) (void)hipFree(m->d_mlp_norm);
    if (m->d_fallbacks) (void)hipFree(m->d_fallbacks);
    if (m->d_hevi_fac) (void)hipFree(m->d_hevi_fac);
    for (auto& r : m->prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    delete m;
    return CM_OK;
}

cm_status cm_model_create(const cm_grid* g, const cm_model_desc* desc, const double* Yref, cm_model** out)
{
    if (!g || !desc || !out) { set_error("cm_model_create: null argument"); return CM_ERR_ARG; }
    *out = nullptr;
    if (desc->nvar != 5 && desc->nvar != 6) { set_error("cm_model_create: nvar must be 5 or 6"); return CM_ERR_UNSUPPORTED; }
    if (desc->precision != CM_FP64 && desc->precision != CM_FP32_BULK) { set_error("cm_model_create: bad precision"); return CM_ERR_ARG; }
    if (desc->closure < 0 || desc->closure > 4) { set_error("cm_model_create: bad closure"); return CM_ERR_ARG; }
    if (desc->flux < 0 || desc->flux > 2) { set_error("cm_model_create: bad numerical flux"); return CM_ERR_ARG; }
    if (desc->ice && desc->nvar == 6 && desc->closure == CM_CLOSURE_MLP) {
        set_error("cm_model_create: the learned closure is not built with the ice phase");
        return CM_ERR_UNSUPPORTED;
    }
    if (desc->flux != CM_FLUX_RUSANOV && desc->nvar != 5) {
        set_error("cm_model_create: Roe and HLLC fluxes are for dry models (nvar = 5) only");
        return CM_ERR_UNSUPPORTED;
    }
    if (desc->closure != CM_CLOSURE_NONE && !(desc->Prt > 0.0)) { set_error("cm_model_create: Prt must be > 0"); return CM_ERR_ARG; }
    if (desc->sponge && !(desc->sp_ztop > desc->sp_zs)) { set_error("cm_model_create: sponge needs z_top > z_s"); return CM_ERR_ARG; }
    if (desc->subsidence && !(desc->sub_ztop > 0.0)) { set_error("cm_model_create: subsidence needs z_top > 0"); return CM_ERR_ARG; }
    CM_TRY_HIP(hipSetDevice(g->device), "hipSetDevice");
    cm_model* m = new (std::nothrow) cm_model();
    if (!m) { set_error("cm_model_create: out of host memory"); return CM_ERR_ALLOC; }
    m->grid = g;
    m->device = g->device;
    m->desc = *desc;
    const int64_t nn = g->n_nodes;
    const int moist = desc->nvar == 6;
    m->nf = 0;
    if (desc->closure != CM_CLOSURE_NONE) {
        m->nf = moist ? 12 : 9;
        if (desc->subsidence) m->nf += moist ? 2 : 1;
    }
    const size_t s = desc->precision == CM_FP64 ? 8 : 4;
    m->Delta = std::cbrt((g->h[0] / 4.0) * (g->h[1] / 4.0) * (g->h[2] / 4.0));
    hipError_t e = hipSuccess;
    const int64_t run = s == 8 ? run_nodes<double>() : run_nodes<float>();
    if (m->nf > 0) e = hipMalloc(&m->d_F2, s * m->nf * g->n_elem * run);
    for (int q = 0; q < 2 && e == hipSuccess && m->nf > 0 && moist; ++q)
        e = hipMalloc(&m->d_T[q], sizeof(double) * 2 * g->n_elem * run_nodes<double>());
    // reference state: per level when the mesh is flat and the background is
    // horizontally uniform, else per node
    m->has_ref = Yref != nullptr;
    std::vector<double> Yr;
    if (e == hipSuccess && Yref) {
        int uniform = g->desc.topo == 0;
        const int nv = desc->nvar;
        if (uniform) {
            const int64_t nlev_stride = (int64_t)g->desc.ne[0] * g->desc.ne[1];
            for (int64_t el = 0; el < g->n_elem && uniform; ++el) {
                int64_t base = (el / nlev_stride) * nlev_stride;  // first element of the same layer
                for (int n = 0; n < NP && uniform; ++n)
                    for (int v = 0; v < nv; ++v) {
                        // nodes sharing (k) level: compare against (ex, ey) = (0, 0) element, same (i, j, k)?
                        // horizontally uniform means independent of i, j, ex, ey
                        int k = n / (NQ * NQ);
                        double a = Yref[v * nn + el * NP + n];
                        double b = Yref[v * nn + base * NP + k * NQ * NQ];
                        if (a != b) { uniform = 0; break; }
                    }
            }
        }
        m->ref_per_node = !uniform;
        const int64_t nref = uniform ? (int64_t)g->desc.ne[2] * NQ : nn;
        Yr.assign((size_t)nv * nref, 0.0);
        for (int64_t r = 0; r < nref; ++r) {
            int64_t src = r;
            if (uniform) {
                int64_t ez = r / NQ, k = r % NQ;
                src = ez * (int64_t)g->desc.ne[0] * g->desc.ne[1] * NP + k * NQ * NQ;
            }
            for (int v = 0; v < nv; ++v) {
                double val = Yref[v * nn + src];
                if (desc->precision == CM_FP32_BULK) val = (double)(float)val;
                Yr[v * nref + r] = val;
            }
        }
        e = hipMalloc(&m->d_pr, sizeof(double) * nref);
        if (e == hipSuccess) e = hipMalloc(&m->d_rhor, sizeof(double) * nref);
    }
    if (e == hipSuccess && !Yref) {
        // no background: p_r = rho_r = 0 (per-level zeros, so the kernels
        // read the reference unconditionally)
        m->ref_per_node = 0;
        const size_t nref = (size_t)g->desc.ne[2] * NQ;
        e = hipMalloc(&m->d_pr, sizeof(double) * nref);
        if (e == hipSuccess) e = hipMalloc(&m->d_rhor, sizeof(double) * nref);
        if (e == hipSuccess) e = hipMemset(m->d_pr, 0, sizeof(double) * nref);
        if (e == hipSuccess) e = hipMemset(m->d_rhor, 0, sizeof(double) * nref);
    }
    if (e == hipSuccess) {
        m->n_partials = DIAG_SCRATCH_RECORDS;
        e = hipMalloc(&m->d_partials, sizeof(double) * 16 * m->n_partials);
    }
    if (e == hipSuccess) e = hipMalloc(&m->d_fallbacks, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(m->d_fallbacks, 0, sizeof(unsigned long long));
    // kernel parameters
    KParams& k = m->kp;
    k.ne0 = g->desc.ne[0]; k.ne1 = g->desc.ne[1]; k.ne2 = g->desc.ne[2];
    k.per0 = g->desc.periodic[0] != 0; k.per1 = g->desc.periodic[1] != 0; k.per2 = g->desc.periodic[2] != 0;
    k.n_elem = (int)g->n_elem;
    k.order = g->d_order;
    k.nn = nn;
    k.nnS = g->n_elem * SRUN;
    k.lo0 = g->desc.lo[0]; k.lo1 = g->desc.lo[1]; k.lo2 = g->desc.lo[2];
    k.h0 = g->h[0]; k.h1 = g->h[1]; k.h2 = g->h[2];
    k.r2h0 = 2.0 / g->h[0]; k.r2h1 = 2.0 / g->h[1]; k.r2h2 = 2.0 / g->h[2];
    k.lift0 = 2.0 / (g->h[0] * g->w[4]); k.lift1 = 2.0 / (g->h[1] * g->w[4]); k.lift2 = 2.0 / (g->h[2] * g->w[4]);
    for (int q = 0; q < NQ; ++q) k.zgll[q] = 0.5 * (1.0 + g->xi[q]);
    k.warped = g->desc.topo == 1;
    k.metrics = desc->precision == CM_FP64 ? (const void*)g->d_metrics64 : (const void*)g->d_metrics32;
    k.zn = g->d_z;
    k.pr = m->d_pr; k.rhor = m->d_rhor;
    k.ref_per_node = m->ref_per_node; k.has_ref = m->has_ref;
    k.g = desc->g;
    k.closure = desc->closure;
    k.nu = desc->nu; k.Cs = desc->Cs; k.Prt = desc->Prt; k.Delta = m->Delta;
    k.invPrt = desc->Prt > 0.0 ? 1.0 / desc->Prt : 0.0;
    k.richardson = desc->richardson != 0;
    k.f_cor = desc->f_cor; k.u_g = desc->u_g; k.v_g = desc->v_g;
    k.sponge = desc->sponge != 0;
    k.sp_zs = desc->sp_zs; k.sp_ztop = desc->sp_ztop; k.sp_alpha = desc->sp_alpha; k.sp_gamma = desc->sp_gamma;
    k.sp_u0 = desc->sp_u[0]; k.sp_u1 = desc->sp_u[1]; k.sp_u2 = desc->sp_u[2];
    k.sp_inv = desc->sponge ? 1.0 / (desc->sp_ztop - desc->sp_zs) : 0.0;
    k.sfc_flux = desc->sfc_flux != 0; k.theta_flux = desc->theta_flux; k.qt_flux = desc->qt_flux;
    k.subsidence = desc->subsidence != 0; k.sub_w0 = desc->sub_w0; k.sub_ztop = desc->sub_ztop;
    k.ice = desc->nvar == 6 && desc->ice != 0;
    k.sub_inv = desc->subsidence ? 1.0 / desc->sub_ztop : 0.0;
    k.nf = m->nf;
    k.nnf = g->n_elem * (desc->precision == CM_FP64 ? run_nodes<double>() : run_nodes<float>());
    k.mlp_frag = nullptr; k.mlp_bias = nullptr; k.mlp_norm = nullptr;
    k.mlp_fallback_on = 1; k.mlp_fallbacks = m->d_fallbacks;
    k.feat_out = nullptr;
    k.Tn = m->d_T[0];
    k.Tnext = nullptr;
    k.T_given = 0;
    k.nnT = g->n_elem * run_nodes<double>();
    if (e == hipSuccess) {
        // the background in conserved variables (kept for the modal filter,
        // which acts on deviations from it), then pushed through the device
        // thermodynamics for p_r and rho_r
        const size_t nref = m->ref_per_node ? (size_t)nn : (size_t)g->desc.ne[2] * NQ;
        m->nref = (int64_t)nref;
        e = hipMalloc(&m->d_Yref, sizeof(double) * desc->nvar * nref);
        if (e == hipSuccess && Yref)
            e = hipMemcpy(m->d_Yref, Yr.data(), sizeof(double) * Yr.size(), hipMemcpyHostToDevice);
        else if (e == hipSuccess)
            e = hipMemset(m->d_Yref, 0, sizeof(double) * desc->nvar * nref);
        if (e == hipSuccess && Yref) e = launch_reference(m, m->d_Yref, nullptr);
        // FP32-bulk states are stored as deviations from the background (its
        // values were rounded to float above, so this copy is exact)
        if (e == hipSuccess && desc->precision == CM_FP32_BULK) {
            std::vector<float> b((size_t)desc->nvar * nref, 0.0f);
            if (Yref)
                for (size_t q = 0; q < b.size(); ++q) b[q] = (float)Yr[q];
            e = hipMalloc(&m->d_bg32, sizeof(float) * b.size());
            if (e == hipSuccess) e = hipMemcpy(m->d_bg32, b.data(), sizeof(float) * b.size(), hipMemcpyHostToDevice);
            if (e == hipSuccess && Yref) {
                // the background as given, in the same table layout
                std::vector<double> b64((size_t)desc->nvar * nref);
                for (int64_t r = 0; r < (int64_t)nref; ++r) {
                    int64_t src = r;
                    if (!m->ref_per_node) {
                        const int64_t ez = r / NQ, k = r % NQ;
                        src = ez * (int64_t)g->desc.ne[0] * g->desc.ne[1] * NP + k * NQ * NQ;
                    }
                    for (int v = 0; v < desc->nvar; ++v) b64[(size_t)v * nref + r] = Yref[(int64_t)v * nn + src];
                }
                e = hipMalloc(&m->d_bg64, sizeof(double) * b64.size());
                if (e == hipSuccess)
                    e = hipMemcpy(m->d_bg64, b64.data(), sizeof(double) * b64.size(), hipMemcpyHostToDevice);
            }
        }
        m->kp.bg32 = m->d_bg32;
        m->kp.nref = m->nref;
        // the 1-D IMEX line factor, for models whose vertical lines all share
        // one matrix (dry, flat mesh, walls at the bottom and top, background
        // per level)
        if (e == hipSuccess && desc->nvar == 5 && g->desc.topo == 0 && !g->desc.periodic[2] && !m->ref_per_node)
            e = hipMalloc(&m->d_hevi_fac, sizeof(double) * hevi_factor_doubles(g->desc.ne[2]));
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    if (e != hipSuccess) {
        cm_status st = hip_fail(e, "cm_model_create");
        cm_model_destroy(m);
        return st;
    }
    *out = m;
    return CM_OK;
}

static cm_status check_model(const cm_model* m, const char* where)
{
    if (!m) { set_error(std::string(where) + ": null model"); return CM_ERR_ARG; }
    if (m->desc.closure == CM_CLOSURE_MLP && !m->mlp_ready) {
        set_error(std::string(where) + ": learned closure selected but no weights set");
        return CM_ERR_STATE;
    }
    return CM_OK;
}

cm_status cm_dg_rhs(cm_model* m, const void* Y, void* dYdt, double t, void* stream)
{
    (void)t;
    cm_status st = check_model(m, "cm_dg_rhs");
    if (st != CM_OK) return st;
    if (!Y || !dYdt) { set_error("cm_dg_rhs: null state pointer"); return CM_ERR_ARG; }
    if (Y == dYdt) { set_error("cm_dg_rhs: Y and dYdt must not alias"); return CM_ERR_ARG; }
    CM_TRY_HIP(hipSetDevice(m->grid->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    CM_TRY_HIP(launch_rhs(m, Y, dYdt, nullptr, 0, 0.0, 0.0, 0.0, s), "cm_dg_rhs launch");
    return CM_OK;
}

// Carpenter & Kennedy (1994) five-stage fourth-order 2N-storage coefficients
static const double LSRK_A[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                                 -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
static const double LSRK_B[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                                 1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                                 2277821191437.0 / 14882151754819.0};

// Niegemann, Diehl & Busch (2012) fourteen-stage fourth-order 2N-storage
// coefficients (sixteen digits, as published)
static const double LSRK144_A[14] = {0.0, -0.7188012108672410, -0.7785331173421570, -0.0053282796654044,
                                     -0.8552979934029281, -3.9564138245774565, -1.5780575380587385,
                                     -2.0837094552574054, -0.7483334182761610, -0.7032861106563359,
                                     0.0013917096117681, -0.0932075369637460, -0.9514200470875948,
                                     -7.1151571693922548};
static const double LSRK144_B[14] = {0.0367762454319673, 0.3136296607553959, 0.1531848691869027,
                                     0.0030097086818182, 0.3326293790646110, 0.2440251405350864,
                                     0.3718879239592277, 0.6204126221582444, 0.1524043173028741,
                                     0.0760894927419266, 0.0077604214040978, 0.0024647284755382,
                                     0.0780348340049386, 5.5059777270269628};

// ns fused stages of a 2N-storage scheme, ping-ponging Y -> Y_alt -> Y ...
static cm_status lsrk_run(cm_model* m, void* Y, void* Y_alt, void* dQ, double dt, int ns, const double* A,
                          const double* B, void* stream, const char* name)
{
    cm_status st = check_model(m, name);
    if (st != CM_OK) return st;
    if (!Y || !Y_alt || !dQ) { set_error(std::string(name) + ": null state pointer"); return CM_ERR_ARG; }
    if (Y == Y_alt || Y == dQ || Y_alt == dQ) { set_error(std::string(name) + ": Y, Y_alt, dQ must be distinct"); return CM_ERR_ARG; }
    if (!(dt > 0.0) || !std::isfinite(dt)) { set_error(std::string(name) + ": dt must be positive and finite"); return CM_ERR_ARG; }
    CM_TRY_HIP(hipSetDevice(m->grid->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    void* src = Y;
    void* dst = Y_alt;
    for (int stage = 0; stage < ns; ++stage) {
        CM_TRY_HIP(launch_rhs(m, src, dst, dQ, stage == 0 ? 2 : 1, A[stage], B[stage], dt, s), name);
        void* tmp = src;
        src = dst;
        dst = tmp;
    }
    return CM_OK;
}

cm_status cm_lsrk_step(cm_model* m, void* Y, void* Y_alt, void* dQ, double t, double dt, void* stream)
{
    (void)t;
    return lsrk_run(m, Y, Y_alt, dQ, dt, 5, LSRK_A, LSRK_B, stream, "cm_lsrk_step");
}

cm_status cm_lsrk144_step(cm_model* m, void* Y, void* Y_alt, void* dQ, double t, double dt, void* stream)
{
    (void)t;
    return lsrk_run(m, Y, Y_alt, dQ, dt, 14, LSRK144_A, LSRK144_B, stream, "cm_lsrk144_step");
}

cm_status cm_model_profile(cm_model* m, int enable)
{
    if (!m) { set_error("cm_model_profile: null model"); return CM_ERR_ARG; }
    m->profiling = enable != 0;
    m->prof_used = 0;
    return CM_OK;
}

cm_status cm_model_profile_read(cm_model* m, double* ms, int64_t* count)
{
    if (!m || !ms || !count) { set_error("cm_model_profile_read: null argument"); return CM_ERR_ARG; }
    ms[0] = ms[1] = 0.0;
    count[0] = count[1] = 0;
    for (size_t q = 0; q < m->prof_used; ++q) {
        const cm_model::ProfRec& r = m->prof[q];
        CM_TRY_HIP(hipEventSynchronize(r.b), "hipEventSynchronize");
        float t = 0.0f;
        CM_TRY_HIP(hipEventElapsedTime(&t, r.a, r.b), "hipEventElapsedTime");
        ms[r.kind] += t;
        count[r.kind] += 1;
    }
    return CM_OK;
}

cm_status cm_model_closure_inputs(cm_model* m, const void* Y, double* feat, void* stream)
{
    if (!m || !Y || !feat) { set_error("cm_model_closure_inputs: null argument"); return CM_ERR_ARG; }
    if (m->desc.closure != CM_CLOSURE_SMAG || !m->desc.richardson) {
        set_error("cm_model_closure_inputs: needs the Smagorinsky closure with the Richardson factor");
        return CM_ERR_STATE;
    }
    if (m->kp.ice) {
        set_error("cm_model_closure_inputs: not built with the ice phase");
        return CM_ERR_UNSUPPORTED;
    }
    CM_TRY_HIP(hipSetDevice(m->grid->device), "hipSetDevice");
    m->kp.feat_out = feat;
    hipError_t e = launch_grad_only(m, Y, (hipStream_t)stream);
    m->kp.feat_out = nullptr;
    CM_TRY_HIP(e, "cm_model_closure_inputs");
    return CM_OK;
}

cm_status cm_diagnostics(cm_model* m, const void* Y, double dt, cm_diag* out, void* stream)
{
    if (!m || !Y || !out) { set_error("cm_diagnostics: null argument"); return CM_ERR_ARG; }
    CM_TRY_HIP(hipSetDevice(m->grid->device), "hipSetDevice");
    CM_TRY_HIP(launch_diagnostics(m, Y, dt, out, (hipStream_t)stream), "cm_diagnostics");
    if (out->n_nonfinite > 0) {
        set_error("cm_diagnostics: state holds non-finite values");
        return CM_ERR_NONFINITE;
    }
    return CM_OK;
}

// 1-D exponential filter matrix V diag(sigma) V^-1 on the GLL nodes, V[i][n]
// = P_n(xi_i) (Legendre polynomials by their three-term recurrence, the
// inverse by Gaussian elimination with partial pivoting)
static void exp_filter_matrix(const double* xi, int order, double alpha, int Nc, double* F)
{
    constexpr int Q = NQ, N = NQ - 1;
    double V[Q][Q];
    for (int i = 0; i < Q; ++i) {
        double pm = 1.0, p = xi[i];
        V[i][0] = 1.0;
        V[i][1] = xi[i];
        for (int n = 1; n < N; ++n) {
            const double pn = ((2 * n + 1) * xi[i] * p - n * pm) / (n + 1);
            pm = p;
            p = pn;
            V[i][n + 1] = p;
        }
    }
    // solve V X = diag(sigma) ... as X = V^-1 column by column: W = V^-1
    double Aug[Q][2 * Q];
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < 2 * Q; ++j) Aug[i][j] = j < Q ? V[i][j] : (j - Q == i ? 1.0 : 0.0);
    for (int c = 0; c < Q; ++c) {
        int piv = c;
        for (int r = c + 1; r < Q; ++r)
            if (std::fabs(Aug[r][c]) > std::fabs(Aug[piv][c])) piv = r;
        for (int j = 0; j < 2 * Q; ++j) std::swap(Aug[c][j], Aug[piv][j]);
        for (int r = c + 1; r < Q; ++r) {
            const double f = Aug[r][c] / Aug[c][c];
            for (int j = c; j < 2 * Q; ++j) Aug[r][j] -= f * Aug[c][j];
        }
    }
    for (int c = Q - 1; c >= 0; --c) {
        for (int j = Q; j < 2 * Q; ++j) {
            double v = Aug[c][j];
            for (int k = c + 1; k < Q; ++k) v -= Aug[c][k] * Aug[k][j];
            Aug[c][j] = v / Aug[c][c];
        }
    }
    double sig[Q];
    for (int n = 0; n < Q; ++n)
        sig[n] = n <= Nc ? 1.0 : std::exp(-alpha * std::pow((double)(n - Nc) / (double)(N - Nc), (double)order));
    for (int i = 0; i < Q; ++i)
        for (int l = 0; l < Q; ++l) {
            double acc = 0.0;
            for (int n = 0; n < Q; ++n) acc += V[i][n] * sig[n] * Aug[n][Q + l];
            F[i * Q + l] = acc;
        }
}

cm_status cm_state_import(cm_model* m, const double* Y_full, void* state, void* stream)
{
    if (!m || !Y_full || !state) { set_error("cm_state_import: null argument"); return CM_ERR_ARG; }
    CM_TRY_HIP(hipSetDevice(m->grid->device), "hipSetDevice");
    CM_TRY_HIP(launch_state_convert(m, Y_full, state, true, (hipStream_t)stream), "cm_state_import");
    return CM_OK;
}

cm_status cm_state_export(cm_model* m, const void* state, double* Y_full, void* stream)
{
    if (!m || !Y_full || !state) { set_error("cm_state_export: null argument"); return CM_ERR_ARG; }
    CM_TRY_HIP(hipSetDevice(m->grid->device), "hipSetDevice");
    CM_TRY_HIP(launch_state_convert(m, state, Y_full, false, (hipStream_t)stream), "cm_state_export");
    return CM_OK;
}

cm_status cm_exp_filter(cm_model* m, void* Y, int var_mask, int order, double alpha, int Nc, void* stream)
{
    if (!m || !Y) { set_error("cm_exp_filter: null argument"); return CM_ERR_ARG; }
    if (var_mask <= 0 || var_mask >= (1 << m->desc.nvar)) { set_error("cm_exp_filter: bad variable mask"); return CM_ERR_ARG; }
    if (order < 1 || !(alpha >= 0.0) || !std::isfinite(alpha) || Nc < 0 || Nc >= NQ - 1) {
        set_error("cm_exp_filter: need order >= 1, finite alpha >= 0 and 0 <= Nc < N");
        return CM_ERR_ARG;
    }
    CM_TRY_HIP(hipSetDevice(m->grid->device), "hipSetDevice");
    double F[NQ * NQ];
    exp_filter_matrix(m->grid->xi, order, alpha, Nc, F);
    CM_TRY_HIP(launch_exp_filter(m, Y, var_mask, F, (hipStream_t)stream), "cm_exp_filter");
    return CM_OK;
}

// ---- 1-D IMEX (HEVI) -----------------------------------------------------
static cm_status hevi_check(const cm_model* m, const char* name)
{
    if (!m) { set_error(std::string(name) + ": null model"); return CM_ERR_ARG; }
    const cm_grid* g = m->grid;
    if (m->desc.nvar != 5 || g->desc.topo != 0 || g->desc.periodic[2]) {
        set_error(std::string(name) + ": the 1-D IMEX step is for dry models on flat meshes with walls at "
                                      "the bottom and top");
        return CM_ERR_UNSUPPORTED;
    }
    return CM_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// workspace: six state buffers (the stage state, the right-hand sides of the
// three stages and the vertical operator of the first two), then the line
// solver's 60 doubles per element layer and vertical node line, then its
// background table (h_r and c_r per background entry)
constexpr int HEVI_STATE_BUFFERS = 6;
static size_t hevi_state_bytes(const cm_model* m)
{
    const size_t s = m->desc.precision == CM_FP64 ? 8 : 4;
    return align256(s * m->desc.nvar * m->grid->n_elem * SRUN);
}

cm_status cm_hevi_workspace_bytes(const cm_model* m, size_t* bytes)
{
    cm_status st = hevi_check(m, "cm_hevi_workspace_bytes");
    if (st != CM_OK) return st;
    if (!bytes) { set_error("cm_hevi_workspace_bytes: null argument"); return CM_ERR_ARG; }
    const size_t nref = m->ref_per_node ? (size_t)m->grid->n_nodes : (size_t)m->grid->desc.ne[2] * NQ;
    *bytes = HEVI_STATE_BUFFERS * hevi_state_bytes(m) +
             sizeof(double) * 60 * (size_t)m->grid->desc.ne[2] * (size_t)hevi_lines(m) +
             align256(sizeof(double) * 2 * nref);
    return CM_OK;
}

cm_status cm_hevi_step(cm_model* m, void* Y, void* work, double t, double dt, void* stream)
{
    (void)t;
    cm_status st = hevi_check(m, "cm_hevi_step");
    if (st != CM_OK) return st;
    st = check_model(m, "cm_hevi_step");
    if (st != CM_OK) return st;
    if (!Y || !work) { set_error("cm_hevi_step: null pointer"); return CM_ERR_ARG; }
    if (!(dt > 0.0) || !std::isfinite(dt)) { set_error("cm_hevi_step: dt must be positive and finite"); return CM_ERR_ARG; }
    CM_TRY_HIP(hipSetDevice(m->grid->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const size_t sb = hevi_state_bytes(m);
    char* w = (char*)work;
    void* Ys = w;
    void* Rs[3] = {w + sb, w + 2 * sb, w + 3 * sb};  // R(Y_s), the full right-hand side of each stage
    void* L[2] = {w + 4 * sb, w + 5 * sb};  // L(Y_s), its linear vertical part (the last stage's is not needed)
    double* scratch = (double*)(w + HEVI_STATE_BUFFERS * sb);
    // ARK2 of Giraldo, Kelly & Constantinescu (2013), explicit part R - L,
    // implicit part L: a stage combines a_sr (R_r - L_r) + ahat_sr L_r =
    // a_sr R_r + (ahat_sr - a_sr) L_r, and the weights of the two parts are
    // equal, so the update needs only the R_r
    const double gam = 1.0 - 1.0 / std::sqrt(2.0), del = 1.0 / (2.0 * std::sqrt(2.0));
    const double a32 = (3.0 + 2.0 * std::sqrt(2.0)) / 6.0;
    const double AE[3][3] = {{0, 0, 0}, {2 * gam, 0, 0}, {1 - a32, a32, 0}};
    const double AI[3][3] = {{0, 0, 0}, {gam, gam, 0}, {del, del, gam}};
    const double bw[3] = {del, del, gam};
    for (int stg = 0; stg < 3; ++stg) {
        // the first stage is the state itself
        const void* Yst = stg == 0 ? Y : Ys;
        if (stg > 0) {
            double c[6];
            const void* X[6];
            int n = 0;
            for (int r = 0; r < stg; ++r) {
                c[n] = dt * AE[stg][r]; X[n++] = Rs[r];
                c[n] = dt * (AI[stg][r] - AE[stg][r]); X[n++] = L[r];
            }
            CM_TRY_HIP(launch_combine(m, Y, Ys, n, c, X, s), "cm_hevi_step combine");
            CM_TRY_HIP(launch_hevi_solve(m, dt * AI[stg][stg], Ys, Ys, scratch, s), "cm_hevi_step solve");
        }
        CM_TRY_HIP(launch_rhs(m, Yst, Rs[stg], nullptr, 0, 0.0, 0.0, 0.0, s), "cm_hevi_step rhs");
        if (stg < 2) CM_TRY_HIP(launch_hevi_operator(m, Yst, L[stg], nullptr, s), "cm_hevi_step operator");
    }
    double c[3];
    const void* X[3];
    for (int r = 0; r < 3; ++r) {
        c[r] = dt * bw[r];
        X[r] = Rs[r];
    }
    CM_TRY_HIP(launch_combine(m, Y, Y, 3, c, X, s), "cm_hevi_step update");
    return CM_OK;
}

cm_status cm_hevi_operator(cm_model* m, const void* Y, void* LY, void* stream)
{
    cm_status st = hevi_check(m, "cm_hevi_operator");
    if (st != CM_OK) return st;
    if (!Y || !LY || Y == LY) { set_error("cm_hevi_operator: bad state pointers"); return CM_ERR_ARG; }
    CM_TRY_HIP(hipSetDevice(m->grid->device), "hipSetDevice");
    CM_TRY_HIP(launch_hevi_operator(m, Y, LY, nullptr, (hipStream_t)stream), "cm_hevi_operator");
    return CM_OK;
}

cm_status cm_hevi_solve(cm_model* m, double tau, const void* B, void* Y, void* work, void* stream)
{
    cm_status st = hevi_check(m, "cm_hevi_solve");
    if (st != CM_OK) return st;
    if (!B || !Y || !work || !(tau >= 0.0) || !std::isfinite(tau)) { set_error("cm_hevi_solve: bad argument"); return CM_ERR_ARG; }
    CM_TRY_HIP(hipSetDevice(m->grid->device), "hipSetDevice");
    double* scratch = (double*)((char*)work + HEVI_STATE_BUFFERS * hevi_state_bytes(m));
    CM_TRY_HIP(launch_hevi_solve(m, tau, B, Y, scratch, (hipStream_t)stream), "cm_hevi_solve");
    return CM_OK;
}

cm_status cm_diagnostics_noalloc(cm_model* m, const void* Y, double dt, cm_diag* out, void* stream)
{
    if (!m || !Y || !out) { set_error("cm_diagnostics_noalloc: null argument"); return CM_ERR_ARG; }
    // the first pass strides over the nodes with at most
    // DIAG_SCRATCH_RECORDS - 1 blocks, so the workspace bounds the block
    // count, not the grid; the node count is bounded by the grid's own limit
    if (m->grid->n_nodes <= 0 || 16 * m->grid->n_nodes >= ((int64_t)1 << 31)) {
        set_error("cm_diagnostics_noalloc: node count outside 1 .. 2^27");
        return CM_ERR_ARG;
    }
    CM_TRY_HIP(hipSetDevice(m->grid->device), "hipSetDevice");
    CM_TRY_HIP(launch_diagnostics_static(m, Y, dt, out, (hipStream_t)stream), "cm_diagnostics_noalloc");
    if (out->n_nonfinite > 0) {
        set_error("cm_diagnostics_noalloc: state holds non-finite values");
        return CM_ERR_NONFINITE;
    }
    return CM_OK;
}

}  // extern "C"
