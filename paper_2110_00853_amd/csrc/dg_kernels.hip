// gfx950 kernels of the DG right-hand side (Sect. 3.1, eq. matrixProblem) and
// the fused LSRK54 stage update (Sect. 3.2).
//
// One element per 128-thread block (two wave64), one GLL node per lane
// (125 of 128 lanes active).  Per stage:
//   k_grad  : thermodynamic recovery -> BR1 auxiliary gradients of
//             (u, v, w, h_tot[, q_t][, theta_v]) from LDS-staged element
//             tiles + centred face lifts -> closure -> diffusive flux F2
//             (nf words per node, SoA) to HBM.
//   k_tend  : thermodynamics -> F = F1 + F2 -> contravariant flux in LDS ->
//             strong-form divergence with the 1-D GLL matrix along
//             xi1/xi2/xi3 -> Rusanov / centred face fluxes with the
//             neighbour's face nodes -> sources -> epilogue (write R, or
//             dQ = A dQ + dt R, Y_new = Y + B dQ).
// State layout [var][element][node], node = i + 5 j + 25 k, coalesced per
// (variable, element) as a 125-word run.  Blocks are mapped to elements so
// that each of the eight XCDs walks one contiguous range of elements.
#include <cmath>

#include "cm_impl.hpp"

namespace cm {

__constant__ double c_D[NQ * NQ];
__constant__ float c_Df[NQ * NQ];

hipError_t upload_constants(const cm_grid* g)
{
    float Df[NQ * NQ];
    for (int q = 0; q < NQ * NQ; ++q) Df[q] = (float)g->D[q];
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_D), g->D, sizeof(double) * NQ * NQ);
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_Df), Df, sizeof(float) * NQ * NQ);
    return e;
}

template <typename R> __device__ __forceinline__ R dmat(int r, int c);
template <> __device__ __forceinline__ double dmat<double>(int r, int c) { return c_D[r * NQ + c]; }
template <> __device__ __forceinline__ float dmat<float>(int r, int c) { return c_Df[r * NQ + c]; }

// GLL end weight w_N = 1/10
constexpr double WN = 0.1;

// ---------------------------------------------------------------------------
// block -> element: blocks are dealt round-robin to the eight XCDs; give each
// XCD one contiguous run of elements so neighbours share its L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int elem_of_block(int b, int n)
{
    const int q = n >> 3;
    if (b < (q << 3)) return (b & 7) * q + (b >> 3);
    return b;
}

__device__ __forceinline__ int nbr_elem(const KParams& P, int ex, int ey, int ez, int dir, int side)
{
    int c0 = ex, c1 = ey, c2 = ez;
    if (dir == 0) {
        c0 += side;
        if (c0 < 0 || c0 >= P.ne0) { if (!P.per0) return -1; c0 = (c0 + P.ne0) % P.ne0; }
    } else if (dir == 1) {
        c1 += side;
        if (c1 < 0 || c1 >= P.ne1) { if (!P.per1) return -1; c1 = (c1 + P.ne1) % P.ne1; }
    } else {
        c2 += side;
        if (c2 < 0 || c2 >= P.ne2) { if (!P.per2) return -1; c2 = (c2 + P.ne2) % P.ne2; }
    }
    return c0 + P.ne0 * (c1 + P.ne1 * c2);
}

__device__ __forceinline__ double node_z(const KParams& P, int e, int ez, int k, int t)
{
    if (P.warped) return P.zn[(int64_t)e * NP + t];
    return P.lo2 + ((double)ez + P.zgll[k]) * P.h2;
}

__device__ __forceinline__ int ref_index(const KParams& P, int e, int ez, int k, int t)
{
    return P.ref_per_node ? e * NP + t : ez * NQ + k;
}

// ---------------------------------------------------------------------------
// thermodynamics (Sects. 2.4-2.6), always FP64
// ---------------------------------------------------------------------------
struct Th {
    double rho, u, v, w, e, qt, T, p, c, h, qv, ql, Rm;
};

__device__ __forceinline__ double pvsat(double T)
{
    // Clausius-Clapeyron integrated with constant heat capacities:
    // p* = p_tr (T/T0)^((c_pv-c_pl)/R_v) exp((L_v0-(c_pv-c_pl)T0)/R_v (1/T0 - 1/T))
    constexpr double dc = Phys::cpv - Phys::cpl;
    return Phys::ptr * exp(dc / Phys::Rv * log(T / Phys::T0) +
                           (Phys::Lv0 - dc * Phys::T0) / Phys::Rv * (1.0 / Phys::T0 - 1.0 / T));
}

// Saturation adjustment: T from (rho, q_t, I) by Newton iteration with the
// analytic derivative dI*/dT; unsaturated air returns T_u directly.
__device__ __forceinline__ void saturation_adjust(double rho, double qt, double I, double& T, double& ql)
{
    const double Tu = Phys::T0 + (I - qt * Phys::Iv0) / ((1.0 - qt) * Phys::cvd + qt * Phys::cvv);
    const double qvs_u = pvsat(Tu) / (rho * Phys::Rv * Tu);
    if (qt <= qvs_u) { T = Tu; ql = 0.0; return; }
    double Tn = Tu;
    for (int it = 0; it < 20; ++it) {
        const double qv = pvsat(Tn) / (rho * Phys::Rv * Tn);
        const double dT = Tn - Phys::T0;
        const double f = (1.0 - qt) * Phys::cvd * dT + qv * (Phys::cvv * dT + Phys::Iv0) + (qt - qv) * Phys::cvl * dT - I;
        const double Lv = Phys::Lv0 + (Phys::cpv - Phys::cpl) * dT;
        const double dqv = qv * (Lv / (Phys::Rv * Tn * Tn) - 1.0 / Tn);
        const double cvm = (1.0 - qt) * Phys::cvd + qv * Phys::cvv + (qt - qv) * Phys::cvl;
        const double fp = cvm + dqv * (Phys::Iv0 + (Phys::cvv - Phys::cvl) * dT);
        const double step = f / fp;
        Tn -= step;
        if (fabs(step) <= 1e-13 * Tn) break;
    }
    double qv = pvsat(Tn) / (rho * Phys::Rv * Tn);
    qv = qv < qt ? qv : qt;
    T = Tn;
    ql = qt - qv;
}

template <bool MOIST>
__device__ __forceinline__ void thermo(double rho, double mx, double my, double mz, double re, double rq, double z,
                                       double g, Th& o)
{
    const double ir = 1.0 / rho;
    o.rho = rho;
    o.u = mx * ir; o.v = my * ir; o.w = mz * ir;
    o.e = re * ir;
    const double I = o.e - 0.5 * (o.u * o.u + o.v * o.v + o.w * o.w) - g * z;
    if (MOIST) {
        o.qt = rq * ir;
        saturation_adjust(rho, o.qt, I, o.T, o.ql);
        o.qv = o.qt - o.ql;
        o.Rm = Phys::Rd * (1.0 - o.qt) + Phys::Rv * o.qv;
        const double cvm = (1.0 - o.qt) * Phys::cvd + o.qv * Phys::cvv + o.ql * Phys::cvl;
        o.p = rho * o.Rm * o.T;
        o.c = sqrt((cvm + o.Rm) / cvm * o.Rm * o.T);
    } else {
        o.qt = 0.0; o.ql = 0.0; o.qv = 0.0;
        o.T = Phys::T0 + I * (1.0 / Phys::cvd);
        o.Rm = Phys::Rd;
        o.p = rho * Phys::Rd * o.T;
        o.c = sqrt(Phys::cpd / Phys::cvd * Phys::Rd * o.T);
    }
    o.h = o.e + o.p * ir;
}

// virtual potential temperature theta_v = T (p0/p)^(R_d/c_pd) R_m/R_d
__device__ __forceinline__ double theta_v(const Th& o)
{
    return o.T * exp(Phys::kappa * log(Phys::p0 / o.p)) * (o.Rm / Phys::Rd);
}

// ---------------------------------------------------------------------------
// reference state: background pushed through the same thermodynamics
// ---------------------------------------------------------------------------
template <bool MOIST>
__global__ void k_reference(KParams P, const double* __restrict__ Yr, int64_t nref, double* __restrict__ pr,
                            double* __restrict__ rhor)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nref) return;
    double z;
    if (!P.ref_per_node) {
        const int ez = (int)(r / NQ), k = (int)(r % NQ);
        z = P.lo2 + ((double)ez + P.zgll[k]) * P.h2;
    } else {
        const int e = (int)(r / NP), t = (int)(r % NP);
        const int ez = e / (P.ne0 * P.ne1);
        z = node_z(P, e, ez, t / (NQ * NQ), t);
    }
    Th th;
    thermo<MOIST>(Yr[r], Yr[nref + r], Yr[2 * nref + r], Yr[3 * nref + r], Yr[4 * nref + r],
                  MOIST ? Yr[5 * nref + r] : 0.0, z, P.g, th);
    pr[r] = th.p;
    rhor[r] = th.rho;
}

hipError_t launch_reference(const cm_model* m, const double* Yr, hipStream_t s)
{
    const int64_t nref = m->ref_per_node ? m->grid->n_nodes : (int64_t)m->grid->desc.ne[2] * NQ;
    const int nb = (int)((nref + 255) / 256);
    if (m->desc.nvar == 6)
        hipLaunchKernelGGL(k_reference<true>, dim3(nb), dim3(256), 0, s, m->kp, Yr, nref, m->d_pr, m->d_rhor);
    else
        hipLaunchKernelGGL(k_reference<false>, dim3(nb), dim3(256), 0, s, m->kp, Yr, nref, m->d_pr, m->d_rhor);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// metric helpers
// ---------------------------------------------------------------------------
template <typename R>
struct Metric {
    R Ja[3][3];
    R invJ;
};

template <typename R, bool WARP>
__device__ __forceinline__ void load_metric(const KParams& P, int64_t node, Metric<R>& M)
{
    if (WARP) {
        const R* m = (const R*)P.metrics;
#pragma unroll
        for (int q = 0; q < 9; ++q) M.Ja[q / 3][q % 3] = m[(int64_t)q * P.nn + node];
        M.invJ = m[9 * P.nn + node];
    }
}

// face normal, |J^s| and lift factor J^s/(J w_N) at a node of face (dir, side)
template <typename R, bool WARP>
__device__ __forceinline__ void face_geom(const KParams& P, const Metric<R>& M, int dir, int side, R n[3], R& lift)
{
    if (WARP) {
        const R a0 = M.Ja[dir][0], a1 = M.Ja[dir][1], a2 = M.Ja[dir][2];
        const R Js = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
        const R inv = (R)side / Js;
        n[0] = a0 * inv; n[1] = a1 * inv; n[2] = a2 * inv;
        lift = Js * M.invJ * (R)(1.0 / WN);
    } else {
        n[0] = n[1] = n[2] = (R)0;
        n[dir] = (R)side;
        const double h = dir == 0 ? P.h0 : (dir == 1 ? P.h1 : P.h2);
        lift = (R)(2.0 / (h * WN));
    }
}

// ---------------------------------------------------------------------------
// Smagorinsky-Lilly with the Richardson stability factor (eq. smago,
// eq. richardson), |S|^2 = 2 S_ij S_ij
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R smagorinsky(const KParams& P, const R S[3][3], R N2)
{
    R SS = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) SS += (R)2 * S[a][b] * S[a][b];
    if (!(SS > (R)0)) return (R)0;
    R fb = (R)1;
    if (P.richardson) {
        const R Ri = N2 / SS;
        if (Ri > (R)0) {
            R a = (R)1 - Ri / (R)P.Prt;
            a = a > (R)0 ? a : (R)0;
            fb = sqrt(sqrt(a));
        }
    }
    const R cd = (R)(P.Cs * P.Delta);
    return cd * cd * sqrt(SS) * fb;
}

// ---------------------------------------------------------------------------
// gradient + closure pass
// ---------------------------------------------------------------------------
template <typename R, bool MOIST, bool WARP>
__global__ __launch_bounds__(BLOCK) void k_grad(const KParams P, const R* __restrict__ Y, R* __restrict__ F2)
{
    constexpr int NV = MOIST ? 6 : 5;
    constexpr int NG = MOIST ? 6 : 5;  // u v w h [qt] thv
    constexpr int GQ = 4, GT = MOIST ? 5 : 4;
    __shared__ R sg[NG][BLOCK];

    const int e = elem_of_block(blockIdx.x, P.n_elem);
    const int t = threadIdx.x;
    const bool act = t < NP;
    const int tt = act ? t : NP - 1;
    const int i = tt % NQ, j = (tt / NQ) % NQ, k = tt / (NQ * NQ);
    const int ex = e % P.ne0, ey = (e / P.ne0) % P.ne1, ez = e / (P.ne0 * P.ne1);
    const int64_t nn = P.nn;
    const int64_t node = (int64_t)e * NP + tt;
    const bool need_thv = (P.closure == CM_CLOSURE_SMAG && P.richardson) || P.closure == CM_CLOSURE_MLP;

    double Yv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Yv[v] = (double)Y[v * nn + node];
    const double z = node_z(P, e, ez, k, tt);
    Th th;
    thermo<MOIST>(Yv[0], Yv[1], Yv[2], Yv[3], Yv[4], MOIST ? Yv[5] : 0.0, z, P.g, th);
    R gm[NG];
    gm[0] = (R)th.u; gm[1] = (R)th.v; gm[2] = (R)th.w; gm[3] = (R)th.h;
    if (MOIST) gm[GQ] = (R)th.qt;
    gm[GT] = need_thv ? (R)theta_v(th) : (R)0;
#pragma unroll
    for (int q = 0; q < NG; ++q) sg[q][t] = gm[q];
    __syncthreads();

    Metric<R> M;
    load_metric<R, WARP>(P, node, M);
    R gr[NG][3];
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        R d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
        for (int l = 0; l < NQ; ++l) {
            d0 += dmat<R>(i, l) * sg[q][l + NQ * (j + NQ * k)];
            d1 += dmat<R>(j, l) * sg[q][i + NQ * (l + NQ * k)];
            d2 += dmat<R>(k, l) * sg[q][i + NQ * (j + NQ * l)];
        }
        if (WARP) {
#pragma unroll
            for (int c = 0; c < 3; ++c) gr[q][c] = M.invJ * (M.Ja[0][c] * d0 + M.Ja[1][c] * d1 + M.Ja[2][c] * d2);
        } else {
            gr[q][0] = (R)(2.0 / P.h0) * d0;
            gr[q][1] = (R)(2.0 / P.h1) * d1;
            gr[q][2] = (R)(2.0 / P.h2) * d2;
        }
    }

    // centred BR1 lifts on faces with a neighbour (walls: g* = g^-)
    const int idx[3] = {i, j, k};
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
#pragma unroll
        for (int sd = 0; sd < 2; ++sd) {
            const int side = sd ? 1 : -1;
            if (idx[dir] != (sd ? NQ - 1 : 0)) continue;
            const int en = nbr_elem(P, ex, ey, ez, dir, side);
            if (en < 0) continue;
            int m3[3] = {i, j, k};
            m3[dir] = sd ? 0 : NQ - 1;
            const int tn = m3[0] + NQ * (m3[1] + NQ * m3[2]);
            const int64_t np = (int64_t)en * NP + tn;
            double Yp[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) Yp[v] = (double)Y[v * nn + np];
            const int ezn = en / (P.ne0 * P.ne1);
            const double zp = node_z(P, en, ezn, m3[2], tn);
            Th tp;
            thermo<MOIST>(Yp[0], Yp[1], Yp[2], Yp[3], Yp[4], MOIST ? Yp[5] : 0.0, zp, P.g, tp);
            R gp[NG];
            gp[0] = (R)tp.u; gp[1] = (R)tp.v; gp[2] = (R)tp.w; gp[3] = (R)tp.h;
            if (MOIST) gp[GQ] = (R)tp.qt;
            gp[GT] = need_thv ? (R)theta_v(tp) : (R)0;
            R n[3], lift;
            face_geom<R, WARP>(P, M, dir, side, n, lift);
#pragma unroll
            for (int q = 0; q < NG; ++q) {
                const R jump = (R)0.5 * (gm[q] + gp[q]) - gm[q];
#pragma unroll
                for (int c = 0; c < 3; ++c) gr[q][c] += lift * jump * n[c];
            }
        }
    }

    // closure and diffusive flux
    R S[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) S[a][b] = (R)0.5 * (gr[a][b] + gr[b][a]);
    R nu = 0, Prt = (R)P.Prt;
    if (P.closure == CM_CLOSURE_CONST) {
        nu = (R)P.nu;
    } else if (P.closure == CM_CLOSURE_SMAG || P.closure == CM_CLOSURE_MLP) {
        const R N2 = P.richardson ? (R)P.g / gm[GT] * gr[GT][2] : (R)0;
        nu = smagorinsky<R>(P, S, N2);
    }
    const R rho = (R)th.rho;
    const R Dt = nu / Prt;
    const R c2 = (R)(-2.0) * rho * nu;
    R w[14] = {};
    w[0] = c2 * S[0][0]; w[1] = c2 * S[1][1]; w[2] = c2 * S[2][2];
    w[3] = c2 * S[0][1]; w[4] = c2 * S[0][2]; w[5] = c2 * S[1][2];
    const R u0 = gm[0], u1 = gm[1], u2 = gm[2];
    const R rDt = rho * Dt;
    w[6] = u0 * w[0] + u1 * w[3] + u2 * w[4] - rDt * gr[3][0];
    w[7] = u0 * w[3] + u1 * w[1] + u2 * w[5] - rDt * gr[3][1];
    w[8] = u0 * w[4] + u1 * w[5] + u2 * w[2] - rDt * gr[3][2];
    if (MOIST) {
        w[9] = -rDt * gr[GQ][0];
        w[10] = -rDt * gr[GQ][1];
        w[11] = -rDt * gr[GQ][2];
    }
    // subsidence needs d/dz of h_tot (and q_t) in the tendency pass
    constexpr int SB = MOIST ? 12 : 9;
    w[SB] = gr[3][2];
    if (MOIST) w[SB + 1] = gr[GQ][2];
    const int nw = SB + (P.subsidence ? (MOIST ? 2 : 1) : 0);
    if (act) {
#pragma unroll
        for (int q = 0; q < 14; ++q)
            if (q < nw) F2[q * nn + node] = w[q];
    }
}

// ---------------------------------------------------------------------------
// tendency pass
// ---------------------------------------------------------------------------
// inviscid flux F1 (momentum carries p - p_r)
template <typename R, bool MOIST>
__device__ __forceinline__ void flux1(const Th& o, double pr, R F[][3])
{
    const R rho = (R)o.rho, u[3] = {(R)o.u, (R)o.v, (R)o.w};
    const R pp = (R)(o.p - pr);
    const R ep = (R)(o.rho * o.e + o.p);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const R m = rho * u[d];
        F[0][d] = m;
        F[1][d] = m * u[0];
        F[2][d] = m * u[1];
        F[3][d] = m * u[2];
        F[4][d] = ep * u[d];
        if (MOIST) F[5][d] = (R)(o.rho * o.qt) * u[d];
    }
    F[1][0] += pp;
    F[2][1] += pp;
    F[3][2] += pp;
}

// normal component of the stored diffusive flux
template <typename R, bool MOIST>
__device__ __forceinline__ void f2_normal(const R* w, const R u[3], const R n[3], R out[])
{
    out[0] = MOIST ? w[9] * n[0] + w[10] * n[1] + w[11] * n[2] : (R)0;
    out[1] = w[0] * n[0] + w[3] * n[1] + w[4] * n[2];
    out[2] = w[3] * n[0] + w[1] * n[1] + w[5] * n[2];
    out[3] = w[4] * n[0] + w[5] * n[1] + w[2] * n[2];
    out[4] = w[6] * n[0] + w[7] * n[1] + w[8] * n[2];
    if (MOIST) {
        out[1] += out[0] * u[0];
        out[2] += out[0] * u[1];
        out[3] += out[0] * u[2];
        out[5] = out[0];
    }
}

// MODE 0: out = R; MODE 1: LSRK stage; MODE 2: first LSRK stage (A = 0, dQ not read)
template <typename R, bool MOIST, bool WARP, bool VISC, int MODE>
__global__ __launch_bounds__(BLOCK) void k_tend(const KParams P, const R* __restrict__ Y, const R* __restrict__ F2,
                                                R* __restrict__ out, R* __restrict__ dQ, R A, R B, R dt)
{
    constexpr int NV = MOIST ? 6 : 5;
    __shared__ R sG[NV * 3][BLOCK];

    const int e = elem_of_block(blockIdx.x, P.n_elem);
    const int t = threadIdx.x;
    const bool act = t < NP;
    const int tt = act ? t : NP - 1;
    const int i = tt % NQ, j = (tt / NQ) % NQ, k = tt / (NQ * NQ);
    const int ex = e % P.ne0, ey = (e / P.ne0) % P.ne1, ez = e / (P.ne0 * P.ne1);
    const int64_t nn = P.nn;
    const int64_t node = (int64_t)e * NP + tt;

    R Yr[NV];
    double Yv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        Yr[v] = Y[v * nn + node];
        Yv[v] = (double)Yr[v];
    }
    const double z = node_z(P, e, ez, k, tt);
    const int ri = ref_index(P, e, ez, k, tt);
    const double pr = P.has_ref ? P.pr[ri] : 0.0;
    const double rr = P.has_ref ? P.rhor[ri] : 0.0;
    Th th;
    thermo<MOIST>(Yv[0], Yv[1], Yv[2], Yv[3], Yv[4], MOIST ? Yv[5] : 0.0, z, P.g, th);
    R F1[NV][3];
    flux1<R, MOIST>(th, pr, F1);
    R w[14];
    const R um[3] = {(R)th.u, (R)th.v, (R)th.w};
    if (VISC) {
        const int nw = (MOIST ? 12 : 9) + (P.subsidence ? (MOIST ? 2 : 1) : 0);
#pragma unroll
        for (int q = 0; q < 14; ++q) {
            if (q < nw) w[q] = F2[q * nn + node];
            else w[q] = (R)0;
        }
    }

    Metric<R> M;
    load_metric<R, WARP>(P, node, M);
    // contravariant total flux J a^d . F (Cartesian: (2/h_d) F_d, J folded)
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        R F[3] = {F1[v][0], F1[v][1], F1[v][2]};
        if (VISC) {
            if (v == 0 && MOIST) { F[0] += w[9]; F[1] += w[10]; F[2] += w[11]; }
            if (v == 1) { F[0] += w[0]; F[1] += w[3]; F[2] += w[4]; }
            if (v == 2) { F[0] += w[3]; F[1] += w[1]; F[2] += w[5]; }
            if (v == 3) { F[0] += w[4]; F[1] += w[5]; F[2] += w[2]; }
            if (v == 4) { F[0] += w[6]; F[1] += w[7]; F[2] += w[8]; }
            if (MOIST && v >= 1 && v <= 3) {
                const R uu = um[v - 1];
                F[0] += w[9] * uu; F[1] += w[10] * uu; F[2] += w[11] * uu;
            }
            if (MOIST && v == 5) { F[0] += w[9]; F[1] += w[10]; F[2] += w[11]; }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            R G;
            if (WARP) G = M.Ja[d][0] * F[0] + M.Ja[d][1] * F[1] + M.Ja[d][2] * F[2];
            else G = (R)(2.0 / (d == 0 ? P.h0 : (d == 1 ? P.h1 : P.h2))) * F[d];
            sG[v * 3 + d][t] = G;
        }
    }
    __syncthreads();

    R Rv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        R s = 0;
#pragma unroll
        for (int l = 0; l < NQ; ++l) {
            s += dmat<R>(i, l) * sG[v * 3 + 0][l + NQ * (j + NQ * k)];
            s += dmat<R>(j, l) * sG[v * 3 + 1][i + NQ * (l + NQ * k)];
            s += dmat<R>(k, l) * sG[v * 3 + 2][i + NQ * (j + NQ * l)];
        }
        Rv[v] = WARP ? -s * M.invJ : -s;
    }

    // faces owned by this element: lift (n.F^- - n.F^*)
    const int idx[3] = {i, j, k};
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
#pragma unroll
        for (int sd = 0; sd < 2; ++sd) {
            const int side = sd ? 1 : -1;
            if (idx[dir] != (sd ? NQ - 1 : 0)) continue;
            R n[3], lift;
            face_geom<R, WARP>(P, M, dir, side, n, lift);
            R fm1[NV], fm2[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) fm1[v] = F1[v][0] * n[0] + F1[v][1] * n[1] + F1[v][2] * n[2];
            if (VISC) f2_normal<R, MOIST>(w, um, n, fm2);
            const R unm = um[0] * n[0] + um[1] * n[1] + um[2] * n[2];
            const int en = nbr_elem(P, ex, ey, ez, dir, side);
            R fstar[NV];
            if (en >= 0) {
                int m3[3] = {i, j, k};
                m3[dir] = sd ? 0 : NQ - 1;
                const int tn = m3[0] + NQ * (m3[1] + NQ * m3[2]);
                const int64_t np = (int64_t)en * NP + tn;
                R Ypr[NV];
                double Yp[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    Ypr[v] = Y[v * nn + np];
                    Yp[v] = (double)Ypr[v];
                }
                const int ezn = en / (P.ne0 * P.ne1);
                const double zp = node_z(P, en, ezn, m3[2], tn);
                const double prp = P.has_ref ? P.pr[ref_index(P, en, ezn, m3[2], tn)] : 0.0;
                Th tp;
                thermo<MOIST>(Yp[0], Yp[1], Yp[2], Yp[3], Yp[4], MOIST ? Yp[5] : 0.0, zp, P.g, tp);
                R Fp[NV][3];
                flux1<R, MOIST>(tp, prp, Fp);
                const R up[3] = {(R)tp.u, (R)tp.v, (R)tp.w};
                const R unp = up[0] * n[0] + up[1] * n[1] + up[2] * n[2];
                const R lm = fabs(unm) + (R)th.c, lp = fabs(unp) + (R)tp.c;
                const R lam = lm > lp ? lm : lp;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const R fp = Fp[v][0] * n[0] + Fp[v][1] * n[1] + Fp[v][2] * n[2];
                    fstar[v] = (R)0.5 * (fm1[v] + fp) + (R)0.5 * lam * (Yr[v] - Ypr[v]);
                }
                if (VISC) {
                    R wp[14];
                    const int nw = MOIST ? 12 : 9;
#pragma unroll
                    for (int q = 0; q < 12; ++q) {
                        if (q < nw) wp[q] = F2[q * nn + np];
                        else wp[q] = (R)0;
                    }
                    R fp2[NV];
                    f2_normal<R, MOIST>(wp, up, n, fp2);
#pragma unroll
                    for (int v = 0; v < NV; ++v) fstar[v] += (R)0.5 * (fm2[v] + fp2[v]);
                }
            } else {
                // reflecting ghost u+ = u- - 2 (n.u-) n; rho, rho e, rho q mirrored
                R Ypr[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) Ypr[v] = Yr[v];
                const double mn = Yv[1] * (double)n[0] + Yv[2] * (double)n[1] + Yv[3] * (double)n[2];
                double Yg[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) Yg[v] = Yv[v];
                Yg[1] = Yv[1] - 2.0 * mn * (double)n[0];
                Yg[2] = Yv[2] - 2.0 * mn * (double)n[1];
                Yg[3] = Yv[3] - 2.0 * mn * (double)n[2];
                Ypr[1] = (R)Yg[1]; Ypr[2] = (R)Yg[2]; Ypr[3] = (R)Yg[3];
                Th tp;
                thermo<MOIST>(Yg[0], Yg[1], Yg[2], Yg[3], Yg[4], MOIST ? Yg[5] : 0.0, z, P.g, tp);
                R Fp[NV][3];
                flux1<R, MOIST>(tp, pr, Fp);
                const R up[3] = {(R)tp.u, (R)tp.v, (R)tp.w};
                const R unp = up[0] * n[0] + up[1] * n[1] + up[2] * n[2];
                const R lm = fabs(unm) + (R)th.c, lp = fabs(unp) + (R)tp.c;
                const R lam = lm > lp ? lm : lp;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const R fp = Fp[v][0] * n[0] + Fp[v][1] * n[1] + Fp[v][2] * n[2];
                    fstar[v] = (R)0.5 * (fm1[v] + fp) + (R)0.5 * lam * (Yr[v] - Ypr[v]);
                }
                if (VISC && P.sfc_flux && dir == 2 && sd == 0) {
                    // prescribed upward surface fluxes; the outward normal is -z
                    const double qf = MOIST ? P.qt_flux : 0.0;
                    fstar[4] += (R)(-th.rho * (Phys::cpd * P.theta_flux + Phys::Lv0 * qf));
                    if (MOIST) {
                        fstar[0] += (R)(-th.rho * qf);
                        fstar[5] += (R)(-th.rho * qf);
                    }
                }
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const R fm = VISC ? fm1[v] + fm2[v] : fm1[v];
                Rv[v] += lift * (fm - fstar[v]);
            }
        }
    }

    // sources
    Rv[3] -= (R)((th.rho - rr) * P.g);
    if (P.f_cor != 0.0) {
        Rv[1] += (R)(P.f_cor * (Yv[2] - th.rho * P.v_g));
        Rv[2] -= (R)(P.f_cor * (Yv[1] - th.rho * P.u_g));
    }
    if (P.sponge && z > P.sp_zs) {
        const double zeta = (z - P.sp_zs) / (P.sp_ztop - P.sp_zs);
        const double tau = P.sp_alpha * pow(sin(0.5 * M_PI * zeta), P.sp_gamma);
        Rv[1] -= (R)(tau * (Yv[1] - th.rho * P.sp_u0));
        Rv[2] -= (R)(tau * (Yv[2] - th.rho * P.sp_u1));
        Rv[3] -= (R)(tau * (Yv[3] - th.rho * P.sp_u2));
    }
    if (VISC && P.subsidence) {
        const double zz = z < P.sub_ztop ? z : P.sub_ztop;
        const double ws = -P.sub_w0 * sin(M_PI * zz / P.sub_ztop);
        const int b = MOIST ? 12 : 9;
        Rv[4] -= (R)(th.rho * ws) * w[b];
        if (MOIST) Rv[5] -= (R)(th.rho * ws) * w[b + 1];
    }

    if (!act) return;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int64_t a = v * nn + node;
        if (MODE == 0) {
            out[a] = Rv[v];
        } else {
            const R dq = MODE == 1 ? A * dQ[a] + dt * Rv[v] : dt * Rv[v];
            dQ[a] = dq;
            out[a] = Yr[v] + B * dq;
        }
    }
}

template <typename R, bool MOIST, bool WARP>
static hipError_t launch_typed(cm_model* m, const void* Y, void* out, void* dQ, int mode, double A, double B,
                               double dt, hipStream_t s)
{
    const KParams& P = m->kp;
    const dim3 grid(P.n_elem), block(BLOCK);
    const R* y = (const R*)Y;
    R* F2 = (R*)m->d_F2;
    const bool visc = m->desc.closure != CM_CLOSURE_NONE;
    if (visc) {
        cm_model::ProfRec* r = prof_begin(m, 0, s);
        hipLaunchKernelGGL((k_grad<R, MOIST, WARP>), grid, block, 0, s, P, y, F2);
        prof_end(r, s);
    }
    cm_model::ProfRec* rt = prof_begin(m, 1, s);
#define CM_TEND(V, MD)                                                                                      \
    hipLaunchKernelGGL((k_tend<R, MOIST, WARP, V, MD>), grid, block, 0, s, P, y, (const R*)F2, (R*)out, (R*)dQ, \
                       (R)A, (R)B, (R)dt)
    if (visc) {
        if (mode == 0) CM_TEND(true, 0);
        else if (mode == 1) CM_TEND(true, 1);
        else CM_TEND(true, 2);
    } else {
        if (mode == 0) CM_TEND(false, 0);
        else if (mode == 1) CM_TEND(false, 1);
        else CM_TEND(false, 2);
    }
#undef CM_TEND
    prof_end(rt, s);
    return hipGetLastError();
}

hipError_t launch_rhs(cm_model* m, const void* Y, void* out, void* dQ, int mode, double A, double B, double dt,
                      hipStream_t s)
{
    const bool moist = m->desc.nvar == 6;
    const bool warp = m->grid->desc.topo == 1;
    const bool fp64 = m->desc.precision == CM_FP64;
#define CM_DISPATCH(R, MO, WA) return launch_typed<R, MO, WA>(m, Y, out, dQ, mode, A, B, dt, s)
    if (fp64) {
        if (moist) { if (warp) CM_DISPATCH(double, true, true); else CM_DISPATCH(double, true, false); }
        else { if (warp) CM_DISPATCH(double, false, true); else CM_DISPATCH(double, false, false); }
    } else {
        if (moist) { if (warp) CM_DISPATCH(float, true, true); else CM_DISPATCH(float, true, false); }
        else { if (warp) CM_DISPATCH(float, false, true); else CM_DISPATCH(float, false, false); }
    }
#undef CM_DISPATCH
}

}  // namespace cm
