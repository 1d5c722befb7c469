// 1-D IMEX (HEVI, Sect. 3.2) for dry models on flat meshes: the vertical
// acoustic operator L linearised about the background (DG derivative along
// xi3 with the vertical part of the Rusanov penalty at the background sound
// speed, buoyancy), treated implicitly in the ARK2 step of Giraldo, Kelly &
// Constantinescu; everything else (the full right-hand side minus L)
// explicitly.
//
//   k_vlin   : L (Y - Y_ref) per node, one element per block (fluxes of a
//              vertical node line through LDS, face terms with the element
//              above or below), optionally subtracted from a right-hand side
//   k_vsolve : (I - tau L) x = B - Y_ref on every vertical node line, one
//              line per thread: block-tridiagonal elimination over the
//              element layers with 15 x 15 blocks for (rho, rho w, rho e_tot)
//              (LU with partial pivoting in thread-private LDS), 2 x 2 face
//              systems for the horizontal momenta (only the face penalty
//              couples them)
//   k_combine: out = base + sum_i c_i X_i over the node slots
#include <cmath>

#include "cm_impl.hpp"
#include "fp64_math.hpp"

namespace cm {

struct HeviArgs {
    int ne0, ne1, ne2, ne01;
    int64_t nnS;               // state stride
    int64_t nref;              // background entries per variable
    int ref_per_node;
    const double* Yref;        // [nvar][nref] background, conserved
    const double* pr;          // background pressure [nref]
    double lo2, h2, g, tau;
    double zg[NQ], D[NQ * NQ];
    double* scratch;           // solver workspace [nz][60][n_lines]
};

__device__ __forceinline__ int64_t href(const HeviArgs& A, int e, int ez, int k, int t)
{
    return A.ref_per_node ? (int64_t)e * NP + t : (int64_t)ez * NQ + k;
}

// what a stored state value is relative to: FP64 states hold full values,
// FP32-bulk states their deviation from the background
template <typename R>
__device__ __forceinline__ double sref(const HeviArgs& A, int v, int64_t ri)
{
    if constexpr (sizeof(R) == 8) return A.Yref[v * A.nref + ri];
    else return 0.0;
}

// background quantities at one node: rho_r, p_r, h_r = (E_r + p_r)/rho_r,
// b = R_d T0 - (R_d/c_vd) g z (the coefficient of rho' in p'), c_r
struct HRef {
    double rr, h, b, c;
};

__device__ __forceinline__ HRef href_at(const HeviArgs& A, int64_t ri, int ez, int k)
{
    HRef r;
    r.rr = A.Yref[ri];
    const double pr = A.pr[ri];
    r.h = (A.Yref[4 * A.nref + ri] + pr) * frcp(r.rr);
    const double z = A.lo2 + ((double)ez + A.zg[k]) * A.h2;
    r.b = Phys::Rd * Phys::T0 - (Phys::Rd / Phys::cvd) * A.g * z;
    r.c = fsqrt(Phys::cpd / Phys::cvd * pr * frcp(r.rr));
    return r;
}

// Lout = L (Y - Y_ref); with Eout, also Eout -= Lout (Eout holds R(Y))
template <typename R>
__global__ __launch_bounds__(BLOCK) void k_vlin(const HeviArgs A, const R* __restrict__ Y, R* __restrict__ Lout,
                                                R* __restrict__ Eout)
{
    __shared__ double sF[3][BLOCK];  // vertical fluxes of rho, rho w, rho e_tot
    const int e = blockIdx.x;
    const int t = threadIdx.x;
    const bool act = t < NP;
    const int tt = act ? t : NP - 1;
    const int i = tt % NQ, j = (tt / NQ) % NQ, k = tt / (NQ * NQ);
    const int ez = e / A.ne01;
    const double a = Phys::Rd / Phys::cvd;
    const int64_t soff = (int64_t)e * SRUN + tt;
    const int64_t ri = href(A, e, ez, k, tt);
    const HRef r = href_at(A, ri, ez, k);
    double d[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) d[v] = (double)Y[v * A.nnS + soff] - sref<R>(A, v, ri);
    const double Fm[5] = {d[3], 0.0, 0.0, a * d[4] + r.b * d[0], r.h * d[3]};
    sF[0][t] = Fm[0];
    sF[1][t] = Fm[3];
    sF[2][t] = Fm[4];
    __syncthreads();
    double L[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const double r2h = 2.0 / A.h2;
#pragma unroll
    for (int l = 0; l < NQ; ++l) {
        const double Dkl = A.D[k * NQ + l];
        const int n = i + NQ * (j + NQ * l);
        L[0] -= r2h * Dkl * sF[0][n];
        L[3] -= r2h * Dkl * sF[1][n];
        L[4] -= r2h * Dkl * sF[2][n];
    }
    L[3] -= A.g * d[0];
    if (k == 0 || k == NQ - 1) {
        const double nrm = k == 0 ? -1.0 : 1.0;
        const double lift = r2h * 10.0;  // (2/h_z) / w_N, w_N = 1/10
        const int ezn = ez + (k == 0 ? -1 : 1);
        if (ezn >= 0 && ezn < A.ne2) {
            const int en = e + (k == 0 ? -A.ne01 : A.ne01);
            const int kn = NQ - 1 - k;
            const int tn = i + NQ * (j + NQ * kn);
            const int64_t rin = href(A, en, ezn, kn, tn);
            const HRef rn = href_at(A, rin, ezn, kn);
            double dp[5];
#pragma unroll
            for (int v = 0; v < 5; ++v)
                dp[v] = (double)Y[v * A.nnS + (int64_t)en * SRUN + tn] - sref<R>(A, v, rin);
            const double Fp[5] = {dp[3], 0.0, 0.0, a * dp[4] + rn.b * dp[0], rn.h * dp[3]};
            const double lam = r.c > rn.c ? r.c : rn.c;
#pragma unroll
            for (int v = 0; v < 5; ++v) L[v] += lift * (0.5 * nrm * (Fm[v] - Fp[v]) - 0.5 * lam * (d[v] - dp[v]));
        } else {
            // wall: mirrored ghost (m^+ = -m^-)
            L[0] += lift * nrm * d[3];
            L[3] -= lift * r.c * d[3];
            L[4] += lift * nrm * r.h * d[3];
        }
    }
    if (act) {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            Lout[v * A.nnS + soff] = (R)L[v];
            if (Eout) Eout[v * A.nnS + soff] = (R)((double)Eout[v * A.nnS + soff] - L[v]);
        }
    }
}

constexpr int VS_THREADS = 32;  // lines per block of the line solver
constexpr int VS_N = 15;        // unknowns per element block: (rho, rho w, rho e_tot) x 5 nodes

// LU with partial pivoting of the thread's 15 x 15 block (thread-private
// LDS, the thread index fastest), then solves for nr right-hand sides
__device__ __forceinline__ void lu_solve(double (*M)[VS_N][VS_THREADS], double (*Bm)[4][VS_THREADS], int nr, int t)
{
    for (int c = 0; c < VS_N; ++c) {
        int piv = c;
        double best = fabs(M[c][c][t]);
        for (int r = c + 1; r < VS_N; ++r) {
            const double v = fabs(M[r][c][t]);
            if (v > best) { best = v; piv = r; }
        }
        if (piv != c) {
            for (int q = 0; q < VS_N; ++q) {
                const double tmp = M[c][q][t];
                M[c][q][t] = M[piv][q][t];
                M[piv][q][t] = tmp;
            }
            for (int q = 0; q < nr; ++q) {
                const double tmp = Bm[c][q][t];
                Bm[c][q][t] = Bm[piv][q][t];
                Bm[piv][q][t] = tmp;
            }
        }
        const double inv = 1.0 / M[c][c][t];
        for (int r = c + 1; r < VS_N; ++r) {
            const double f = M[r][c][t] * inv;
            if (f == 0.0) continue;
            for (int q = c + 1; q < VS_N; ++q) M[r][q][t] -= f * M[c][q][t];
            for (int q = 0; q < nr; ++q) Bm[r][q][t] -= f * Bm[c][q][t];
        }
    }
    for (int r = VS_N - 1; r >= 0; --r) {
        const double inv = 1.0 / M[r][r][t];
        for (int q = 0; q < nr; ++q) {
            double v = Bm[r][q][t];
            for (int c = r + 1; c < VS_N; ++c) v -= M[r][c][t] * Bm[c][q][t];
            Bm[r][q][t] = v * inv;
        }
    }
}

// index of (variable 0 rho, 1 rho w, 2 rho e_tot; node k) in an element block
__device__ __forceinline__ int vb(int v3, int k) { return v3 * NQ + k; }

// Jacobian of the vertical flux (rho w, p', h rho w') w.r.t. (rho', m, E')
__device__ __forceinline__ void flux_jac(const HRef& r, double J[3][3])
{
    J[0][0] = 0.0; J[0][1] = 1.0; J[0][2] = 0.0;
    J[1][0] = r.b; J[1][1] = 0.0; J[1][2] = Phys::Rd / Phys::cvd;
    J[2][0] = 0.0; J[2][1] = r.h; J[2][2] = 0.0;
}

// Y_out = Y_ref + x with (I - tau L) x = B - Y_ref on every vertical line
// (B and Y_out may be the same buffer: each thread reads its line before it
// writes it)
template <typename R>
__global__ __launch_bounds__(VS_THREADS) void k_vsolve(const HeviArgs A, const R* __restrict__ B, R* __restrict__ Yo,
                                                       int64_t n_lines)
{
    __shared__ double sM[VS_N][VS_N][VS_THREADS];
    __shared__ double sB[VS_N][4][VS_THREADS];
    const int t = threadIdx.x;
    const int64_t line = (int64_t)blockIdx.x * VS_THREADS + t;
    if (line >= n_lines) return;  // no barriers below: the threads work alone
    const int node = (int)(line % (NQ * NQ));
    const int64_t col = line / (NQ * NQ);
    const int i = node % NQ, j = node / NQ;
    const int ex = (int)(col % A.ne0), ey = (int)(col / A.ne0);
    const double tau = A.tau, r2h = 2.0 / A.h2, lift = r2h * 10.0;
    const int nz = A.ne2;
    double* scr = A.scratch;
    // scratch layout [ez][q][line]: q < 45 the columns of Z_e (15 x 3),
    // 45 .. 59 the forward solution y_e
    auto S = [&](int ez, int q) -> double& { return scr[((int64_t)ez * 60 + q) * n_lines + line]; };
    double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // S_{e-1} Btil_{e-1}
    double yprev[3] = {0, 0, 0};                          // y_{e-1} at its top nodes
    double Cb[3][3];                                      // coupling of this element's bottom to the one below
    for (int ez = 0; ez < nz; ++ez) {
        const int e = ex + A.ne0 * (ey + A.ne1 * ez);
        HRef rk[NQ];
#pragma unroll
        for (int k = 0; k < NQ; ++k) rk[k] = href_at(A, href(A, e, ez, k, i + NQ * (j + NQ * k)), ez, k);
        // assemble I - tau L_e
        for (int r = 0; r < VS_N; ++r)
            for (int c = 0; c < VS_N; ++c) sM[r][c][t] = r == c ? 1.0 : 0.0;
        for (int k = 0; k < NQ; ++k) {
            for (int l = 0; l < NQ; ++l) {
                const double cf = tau * r2h * A.D[k * NQ + l];
                double J[3][3];
                flux_jac(rk[l], J);
                for (int v = 0; v < 3; ++v)
                    for (int w = 0; w < 3; ++w)
                        if (J[v][w] != 0.0) sM[vb(v, k)][vb(w, l)][t] += cf * J[v][w];
            }
            sM[vb(1, k)][vb(0, k)][t] += tau * A.g;
        }
        double Bt[3][3];  // coupling of this element's top to the one above
        for (int side = 0; side < 2; ++side) {
            const int k = side == 0 ? 0 : NQ - 1;
            const double nrm = side == 0 ? -1.0 : 1.0;
            const int ezn = ez + (side == 0 ? -1 : 1);
            if (ezn >= 0 && ezn < nz) {
                const int kn = NQ - 1 - k;
                const int en = e + (side == 0 ? -A.ne01 : A.ne01);
                const HRef rn = href_at(A, href(A, en, ezn, kn, i + NQ * (j + NQ * kn)), ezn, kn);
                const double lam = rk[k].c > rn.c ? rk[k].c : rn.c;
                double Jm[3][3], Jp[3][3];
                flux_jac(rk[k], Jm);
                flux_jac(rn, Jp);
                for (int v = 0; v < 3; ++v)
                    for (int w = 0; w < 3; ++w) {
                        // own node: L += lift (n/2 J^- - lam/2 I); neighbour: L += lift (-n/2 J^+ + lam/2 I)
                        sM[vb(v, k)][vb(w, k)][t] -= tau * lift * (0.5 * nrm * Jm[v][w] - (v == w ? 0.5 * lam : 0.0));
                        const double off = -tau * lift * (-0.5 * nrm * Jp[v][w] + (v == w ? 0.5 * lam : 0.0));
                        if (side == 0) Cb[v][w] = off;
                        else Bt[v][w] = off;
                    }
            } else {
                // wall: L_rho += lift n m, L_m -= lift c m, L_E += lift n h m
                sM[vb(0, k)][vb(1, k)][t] -= tau * lift * nrm;
                sM[vb(1, k)][vb(1, k)][t] += tau * lift * rk[k].c;
                sM[vb(2, k)][vb(1, k)][t] -= tau * lift * nrm * rk[k].h;
                for (int v = 0; v < 3; ++v)
                    for (int w = 0; w < 3; ++w) {
                        if (side == 0) Cb[v][w] = 0.0;
                        else Bt[v][w] = 0.0;
                    }
            }
        }
        // Schur update of the bottom nodes by the elements below
        if (ez > 0)
            for (int v = 0; v < 3; ++v)
                for (int w = 0; w < 3; ++w) {
                    double s = 0.0;
                    for (int q = 0; q < 3; ++q) s += Cb[v][q] * G[q][w];
                    sM[vb(v, 0)][vb(w, 0)][t] -= s;
                }
        // right-hand sides: unit vectors at the top nodes, and the deviation
        for (int r = 0; r < VS_N; ++r) {
            const int v3 = r / NQ, k = r % NQ;
            const int var = v3 == 0 ? 0 : (v3 == 1 ? 3 : 4);
            const int tnode = i + NQ * (j + NQ * k);
            const int64_t ri = href(A, e, ez, k, tnode);
            double rhs = (double)B[var * A.nnS + (int64_t)e * SRUN + tnode] - sref<R>(A, var, ri);
            if (k == 0 && ez > 0) {
                double s = 0.0;
                for (int q = 0; q < 3; ++q) s += Cb[v3][q] * yprev[q];
                rhs -= s;
            }
            sB[r][0][t] = rhs;
            for (int q = 0; q < 3; ++q) sB[r][1 + q][t] = r == vb(q, NQ - 1) ? 1.0 : 0.0;
        }
        lu_solve(sM, sB, 4, t);
        // S_e (3 x 3) = W_e at the top nodes; G = S_e Btil_e; Z_e = W_e Btil_e
        for (int v = 0; v < 3; ++v) {
            for (int w = 0; w < 3; ++w) {
                double s = 0.0;
                for (int q = 0; q < 3; ++q) s += sB[vb(v, NQ - 1)][1 + q][t] * Bt[q][w];
                G[v][w] = s;
            }
            yprev[v] = sB[vb(v, NQ - 1)][0][t];
        }
        for (int r = 0; r < VS_N; ++r) {
            for (int w = 0; w < 3; ++w) {
                double s = 0.0;
                for (int q = 0; q < 3; ++q) s += sB[r][1 + q][t] * Bt[q][w];
                S(ez, r * 3 + w) = s;
            }
            S(ez, 45 + r) = sB[r][0][t];
        }
    }
    // back substitution: x_e = y_e - Z_e x_{e+1}(bottom nodes)
    double xb[3] = {0, 0, 0};
    for (int ez = nz - 1; ez >= 0; --ez) {
        const int e = ex + A.ne0 * (ey + A.ne1 * ez);
        double x[VS_N];
        for (int r = 0; r < VS_N; ++r) {
            double v = S(ez, 45 + r);
            if (ez < nz - 1)
                for (int w = 0; w < 3; ++w) v -= S(ez, r * 3 + w) * xb[w];
            x[r] = v;
        }
        for (int r = 0; r < VS_N; ++r) {
            const int v3 = r / NQ, k = r % NQ;
            const int var = v3 == 0 ? 0 : (v3 == 1 ? 3 : 4);
            const int tnode = i + NQ * (j + NQ * k);
            const int64_t ri = href(A, e, ez, k, tnode);
            Yo[var * A.nnS + (int64_t)e * SRUN + tnode] = (R)(sref<R>(A, var, ri) + x[r]);
        }
        for (int v = 0; v < 3; ++v) xb[v] = x[vb(v, 0)];
    }
    // horizontal momenta: identity except the 2 x 2 systems of the interior
    // vertical faces, [1 + s, -s; -s, 1 + s] with s = tau lift lam / 2
    for (int ez = 0; ez < nz; ++ez) {
        const int e = ex + A.ne0 * (ey + A.ne1 * ez);
        for (int k = 0; k < NQ; ++k) {
            const int tnode = i + NQ * (j + NQ * k);
            const int64_t ri = href(A, e, ez, k, tnode);
            if (k == NQ - 1 && ez < nz - 1) {
                // the pair (top node of ez, bottom node of ez + 1)
                const int en = e + A.ne01;
                const int tn = i + NQ * j;
                const int64_t rin = href(A, en, ez + 1, 0, tn);
                const HRef ra = href_at(A, ri, ez, k), rb = href_at(A, rin, ez + 1, 0);
                const double lam = ra.c > rb.c ? ra.c : rb.c;
                const double s = 0.5 * tau * lift * lam, al = 1.0 + s, det = al * al - s * s;
                for (int v = 1; v <= 2; ++v) {
                    const double xa = (double)B[v * A.nnS + (int64_t)e * SRUN + tnode] - sref<R>(A, v, ri);
                    const double xbv = (double)B[v * A.nnS + (int64_t)en * SRUN + tn] - sref<R>(A, v, rin);
                    Yo[v * A.nnS + (int64_t)e * SRUN + tnode] = (R)(sref<R>(A, v, ri) + (al * xa + s * xbv) / det);
                    Yo[v * A.nnS + (int64_t)en * SRUN + tn] = (R)(sref<R>(A, v, rin) + (s * xa + al * xbv) / det);
                }
            } else if (!(k == 0 && ez > 0)) {
                for (int v = 1; v <= 2; ++v) Yo[v * A.nnS + (int64_t)e * SRUN + tnode] = B[v * A.nnS + (int64_t)e * SRUN + tnode];
            }
        }
    }
}

// out = base + sum_q c_q X_q over the node slots (padding untouched)
struct CombineArgs {
    int n_terms;
    double c[6];
    const void* X[6];
    int64_t n_slots;   // nvar x state stride
};

template <typename R>
__global__ __launch_bounds__(256) void k_combine(const CombineArgs C, const R* __restrict__ base, R* __restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= C.n_slots) return;
    if ((int)(q % SRUN) >= NP) return;
    double v = (double)base[q];
    for (int s = 0; s < C.n_terms; ++s) v += C.c[s] * (double)((const R*)C.X[s])[q];
    out[q] = (R)v;
}

static HeviArgs hevi_args(const cm_model* m, double tau, double* scratch)
{
    const cm_grid* g = m->grid;
    HeviArgs A;
    A.ne0 = g->desc.ne[0];
    A.ne1 = g->desc.ne[1];
    A.ne2 = g->desc.ne[2];
    A.ne01 = A.ne0 * A.ne1;
    A.nnS = g->n_elem * SRUN;
    A.ref_per_node = m->ref_per_node;
    A.nref = m->ref_per_node ? g->n_nodes : (int64_t)g->desc.ne[2] * NQ;
    A.Yref = m->d_Yref;
    A.pr = m->d_pr;
    A.lo2 = g->desc.lo[2];
    A.h2 = g->h[2];
    A.g = m->desc.g;
    A.tau = tau;
    for (int q = 0; q < NQ; ++q) A.zg[q] = 0.5 * (1.0 + g->xi[q]);
    for (int q = 0; q < NQ * NQ; ++q) A.D[q] = g->D[q];
    A.scratch = scratch;
    return A;
}

hipError_t launch_hevi_operator(const cm_model* m, const void* Y, void* Lout, void* Eout, hipStream_t s)
{
    const HeviArgs A = hevi_args(m, 0.0, nullptr);
    const dim3 grid((unsigned)m->grid->n_elem), block(BLOCK);
    if (m->desc.precision == CM_FP64)
        hipLaunchKernelGGL(k_vlin<double>, grid, block, 0, s, A, (const double*)Y, (double*)Lout, (double*)Eout);
    else
        hipLaunchKernelGGL(k_vlin<float>, grid, block, 0, s, A, (const float*)Y, (float*)Lout, (float*)Eout);
    return hipGetLastError();
}

int64_t hevi_lines(const cm_model* m) { return (int64_t)m->grid->desc.ne[0] * m->grid->desc.ne[1] * NQ * NQ; }

hipError_t launch_hevi_solve(const cm_model* m, double tau, const void* B, void* Yout, double* scratch, hipStream_t s)
{
    const HeviArgs A = hevi_args(m, tau, scratch);
    const int64_t nl = hevi_lines(m);
    const dim3 grid((unsigned)((nl + VS_THREADS - 1) / VS_THREADS)), block(VS_THREADS);
    if (m->desc.precision == CM_FP64)
        hipLaunchKernelGGL(k_vsolve<double>, grid, block, 0, s, A, (const double*)B, (double*)Yout, nl);
    else
        hipLaunchKernelGGL(k_vsolve<float>, grid, block, 0, s, A, (const float*)B, (float*)Yout, nl);
    return hipGetLastError();
}

hipError_t launch_combine(const cm_model* m, const void* base, void* out, int n, const double* c, const void* const* X,
                          hipStream_t s)
{
    CombineArgs C;
    C.n_terms = n;
    for (int q = 0; q < n; ++q) { C.c[q] = c[q]; C.X[q] = X[q]; }
    C.n_slots = (int64_t)m->desc.nvar * m->grid->n_elem * SRUN;
    const dim3 grid((unsigned)((C.n_slots + 255) / 256)), block(256);
    if (m->desc.precision == CM_FP64)
        hipLaunchKernelGGL(k_combine<double>, grid, block, 0, s, C, (const double*)base, (double*)out);
    else
        hipLaunchKernelGGL(k_combine<float>, grid, block, 0, s, C, (const float*)base, (float*)out);
    return hipGetLastError();
}

}  // namespace cm
