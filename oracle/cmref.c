/*
 * FP64 CPU oracle for the nodal DG right-hand side, the LSRK54 and LSRK144
 * steps, the 1-D IMEX (HEVI) step, the exponential filter and the
 * conservation integrals.
 *
 * TEST INFRASTRUCTURE ONLY (see cmref.h).  Written as plain loops in the
 * order the paper states the method; correctness over speed.  Parity is
 * pinned by the CPU tests (closed forms, invariants, brute-force dense
 * operators), not by the GPU code.
 *
 * Sections of the paper followed:
 *   Sect. 2 (governing equations, Table 1 constants, EOS, saturation adj.)
 *   Sect. 3.1 (nodal GLL expansion, tensor-product derivatives, mapping,
 *              weak/strong DG form, Rusanov flux, BR1 auxiliary gradient,
 *              semi-discrete matrix problem)
 *   Sect. 2.5, 2.7 and Table 1 (ice phase: liquid fraction, saturation
 *              over the mix)
 *   Sect. 3.1 (Roe and HLLC numerical fluxes for dry air)
 *   Sect. 3.2 (low-storage explicit Runge-Kutta, Carpenter-Kennedy family and
 *              the 14-stage method of Niegemann, Diehl and Busch; additive
 *              Runge-Kutta IMEX with the vertical acoustics implicit)
 *   Sect. 4   (SGS stress, diffusivity, Smagorinsky-Lilly, Richardson corr.,
 *              Vreman eq. vreman-sgs)
 *   Sect. 5.4 (exponential modal filter, eq. exponential_filter)
 *   Sect. 6   (normalised mass / energy integrals)
 *   App. A    (wall ghost states, prescribed wall fluxes, Rayleigh sponge)
 */
#include "cmref.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- constants: Table 1, plus the readings for the values the paper omits
 *      (g, p0, c_pd = c_vd + R_d, triple-point pressure) ------------------- */
static const double RD = 287.0, RV = 462.0;
static const double CVD = 717.5, CVV = 1397.5, CVL = 4181.0;
static const double TREF0 = 273.16;          /* T_0 */
static const double LV0 = 2.5008e6;
static const double P00 = 1.0e5;
static const double PTRIPLE = 611.657;
#define CPD (CVD + RD)
#define CPV (CVV + RV)
#define CPL (CVL)
#define IV0 (LV0 - RV * TREF0)               /* I_{v,0} = L_{v,0} - R_v T_0 */

/* ======================================================================== */
/* GLL nodes, weights and differentiation matrix (Sect. 3.1)                */
/* ======================================================================== */

/* Legendre P_N(x) and its derivative by the three-term recurrence. */
static void legendre(int N, double x, double* P, double* dP)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (N == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int n = 1; n < N; ++n) {
        double p2 = ((2.0 * n + 1.0) * x * p1 - n * p0) / (n + 1.0);
        double d2 = d0 + (2.0 * n + 1.0) * p1;
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *P = p1; *dP = d1;
}

/* Nodes: +-1 and the roots of P_N' (Newton on P_N' using P_N'' from the
 * Legendre ODE).  Weights 2/(N(N+1) P_N(x)^2).  D_ij = l_j'(x_i) from the
 * classical Legendre closed form P_N(x_i)/(P_N(x_j)(x_i-x_j)), i != j, with
 * the diagonal set to minus the off-diagonal row sum. */
int cmref_gll(int N, double* xi, double* w, double* D)
{
    if (N < 1 || N + 1 > CMREF_MAXQ) return 1;
    int Q = N + 1;
    xi[0] = -1.0; xi[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double x = -cos(M_PI * i / N);
        for (int it = 0; it < 100; ++it) {
            double P, dP; legendre(N, x, &P, &dP);
            double d2P = (2.0 * x * dP - N * (N + 1.0) * P) / (1.0 - x * x);
            double dx = dP / d2P;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        xi[i] = x;
    }
    if (N % 2 == 0) xi[N / 2] = 0.0;
    double PN[CMREF_MAXQ];
    for (int i = 0; i < Q; ++i) {
        double P, dP; legendre(N, xi[i], &P, &dP);
        PN[i] = P;
        w[i] = 2.0 / (N * (N + 1.0) * P * P);
    }
    for (int i = 0; i < Q; ++i) {
        double s = 0.0;
        for (int j = 0; j < Q; ++j) {
            if (j == i) continue;
            D[i * Q + j] = PN[i] / (PN[j] * (xi[i] - xi[j]));
            s += D[i * Q + j];
        }
        D[i * Q + i] = -s;
    }
    return 0;
}

/* ======================================================================== */
/* Grid: brick of hexahedra, optional terrain-following warp (Sect. 5.3/5.4) */
/* ======================================================================== */
typedef struct {
    int N, Q, Np;
    int ne[3];
    long nelem, nnodes;
    double lo[3], hi[3], h[3];
    int periodic[3];
    double xi[CMREF_MAXQ], w[CMREF_MAXQ], D[CMREF_MAXQ * CMREF_MAXQ];
    double* xyz;    /* [3][nnodes] */
    double* Ja;     /* [9][nnodes], entry 3*d + c = c-component of J a^d */
    double* J;      /* [nnodes] */
    int dense;      /* apply explicit Kronecker operators for derivatives */
    double* K[3];   /* dense operators Np x Np, built when dense */
} grid_t;

static double agnesi(const cmref_grid_desc* d, double x)
{
    double r = x - d->topo_xc;
    return d->topo_h * d->topo_a * d->topo_a / (r * r + d->topo_a * d->topo_a);
}

/* Reference derivative along direction dir of the nodal field f (element
 * base pointer fe, stride 1 within the element) at local node (i,j,k). */
static double dref(const grid_t* G, const double* fe, int dir, int i, int j, int k)
{
    int Q = G->Q;
    double s = 0.0;
    if (G->dense) {
        int a = i + Q * (j + Q * k);
        const double* row = G->K[dir] + (long)a * G->Np;
        for (int b = 0; b < G->Np; ++b) s += row[b] * fe[b];
        return s;
    }
    if (dir == 0) for (int l = 0; l < Q; ++l) s += G->D[i * Q + l] * fe[l + Q * (j + Q * k)];
    if (dir == 1) for (int l = 0; l < Q; ++l) s += G->D[j * Q + l] * fe[i + Q * (l + Q * k)];
    if (dir == 2) for (int l = 0; l < Q; ++l) s += G->D[k * Q + l] * fe[i + Q * (j + Q * l)];
    return s;
}

void* cmref_grid_create(const cmref_grid_desc* d, int dense)
{
    grid_t* G = (grid_t*)calloc(1, sizeof(grid_t));
    if (!G) return NULL;
    G->N = d->N; G->Q = d->N + 1; G->Np = G->Q * G->Q * G->Q;
    if (cmref_gll(d->N, G->xi, G->w, G->D)) { free(G); return NULL; }
    for (int a = 0; a < 3; ++a) {
        G->ne[a] = d->ne[a]; G->lo[a] = d->lo[a]; G->hi[a] = d->hi[a];
        G->h[a] = (d->hi[a] - d->lo[a]) / d->ne[a]; G->periodic[a] = d->periodic[a];
    }
    G->nelem = (long)d->ne[0] * d->ne[1] * d->ne[2];
    G->nnodes = G->nelem * G->Np;
    long nn = G->nnodes;
    int Q = G->Q, Np = G->Np;
    G->xyz = (double*)malloc(sizeof(double) * 3 * nn);
    G->Ja = (double*)malloc(sizeof(double) * 9 * nn);
    G->J = (double*)malloc(sizeof(double) * nn);
    G->dense = dense;
    if (dense) {
        for (int dir = 0; dir < 3; ++dir) {
            G->K[dir] = (double*)calloc((size_t)Np * Np, sizeof(double));
            for (int k = 0; k < Q; ++k) for (int j = 0; j < Q; ++j) for (int i = 0; i < Q; ++i) {
                int a = i + Q * (j + Q * k);
                for (int l = 0; l < Q; ++l) {
                    int b;
                    if (dir == 0) b = l + Q * (j + Q * k);
                    else if (dir == 1) b = i + Q * (l + Q * k);
                    else b = i + Q * (j + Q * l);
                    G->K[dir][(long)a * Np + b] = G->D[(dir == 0 ? i : dir == 1 ? j : k) * Q + l];
                }
            }
        }
    }
    double ztop = d->hi[2], zlo = d->lo[2];
    /* node coordinates */
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < G->nelem; ++e) {
        int ex = (int)(e % d->ne[0]);
        int ey = (int)((e / d->ne[0]) % d->ne[1]);
        int ez = (int)(e / ((long)d->ne[0] * d->ne[1]));
        for (int k = 0; k < Q; ++k) for (int j = 0; j < Q; ++j) for (int i = 0; i < Q; ++i) {
            long n = e * Np + i + Q * (j + Q * k);
            double x = d->lo[0] + (ex + (1.0 + G->xi[i]) / 2.0) * G->h[0];
            double y = d->lo[1] + (ey + (1.0 + G->xi[j]) / 2.0) * G->h[1];
            double zh = d->lo[2] + (ez + (1.0 + G->xi[k]) / 2.0) * G->h[2];
            double z = zh;
            if (d->topo == 1) z = zh + agnesi(d, x) * (ztop - zh) / (ztop - zlo);
            G->xyz[n] = x; G->xyz[nn + n] = y; G->xyz[2 * nn + n] = z;
        }
    }
    /* metric terms: x_{,xi^d} by D along d; J a^1 = x_eta x x_zeta, ... */
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < G->nelem; ++e) {
        for (int k = 0; k < Q; ++k) for (int j = 0; j < Q; ++j) for (int i = 0; i < Q; ++i) {
            long n = e * Np + i + Q * (j + Q * k);
            double dx[3][3]; /* dx[d][c] = d x_c / d xi^d */
            for (int dir = 0; dir < 3; ++dir)
                for (int c = 0; c < 3; ++c)
                    dx[dir][c] = dref(G, G->xyz + c * nn + e * Np, dir, i, j, k);
            double Ja[3][3];
            for (int dir = 0; dir < 3; ++dir) {
                const double* a = dx[(dir + 1) % 3];
                const double* b = dx[(dir + 2) % 3];
                Ja[dir][0] = a[1] * b[2] - a[2] * b[1];
                Ja[dir][1] = a[2] * b[0] - a[0] * b[2];
                Ja[dir][2] = a[0] * b[1] - a[1] * b[0];
            }
            double Jd = dx[0][0] * Ja[0][0] + dx[0][1] * Ja[0][1] + dx[0][2] * Ja[0][2];
            for (int dir = 0; dir < 3; ++dir)
                for (int c = 0; c < 3; ++c) G->Ja[(3 * dir + c) * nn + n] = Ja[dir][c];
            G->J[n] = Jd;
        }
    }
    return G;
}

void cmref_grid_destroy(void* h)
{
    grid_t* G = (grid_t*)h;
    if (!G) return;
    free(G->xyz); free(G->Ja); free(G->J);
    for (int d = 0; d < 3; ++d) free(G->K[d]);
    free(G);
}

long cmref_grid_nnodes(void* h) { return ((grid_t*)h)->nnodes; }

void cmref_grid_coords(void* h, double* out)
{
    grid_t* G = (grid_t*)h;
    memcpy(out, G->xyz, sizeof(double) * 3 * G->nnodes);
}

void cmref_grid_metrics(void* h, double* Ja, double* J)
{
    grid_t* G = (grid_t*)h;
    memcpy(Ja, G->Ja, sizeof(double) * 9 * G->nnodes);
    memcpy(J, G->J, sizeof(double) * G->nnodes);
}

/* w_i w_j w_k |J| at every node: the collocated (inexact) quadrature weight. */
void cmref_grid_wJ(void* h, double* out)
{
    grid_t* G = (grid_t*)h;
    int Q = G->Q, Np = G->Np;
    for (long e = 0; e < G->nelem; ++e)
        for (int k = 0; k < Q; ++k) for (int j = 0; j < Q; ++j) for (int i = 0; i < Q; ++i) {
            long n = e * Np + i + Q * (j + Q * k);
            out[n] = G->w[i] * G->w[j] * G->w[k] * G->J[n];
        }
}

/* Divergence-of-metrics residual sum_d D_d (J a^d)_c, component c, per node. */
void cmref_grid_metric_identity(void* h, double* out /* [3][nnodes] */)
{
    grid_t* G = (grid_t*)h;
    int Q = G->Q, Np = G->Np; long nn = G->nnodes;
    for (long e = 0; e < G->nelem; ++e)
        for (int k = 0; k < Q; ++k) for (int j = 0; j < Q; ++j) for (int i = 0; i < Q; ++i) {
            long n = e * Np + i + Q * (j + Q * k);
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int dir = 0; dir < 3; ++dir)
                    s += dref(G, G->Ja + (3 * dir + c) * nn + e * Np, dir, i, j, k);
                out[c * nn + n] = s;
            }
        }
}

/* Neighbour of element (ex,ey,ez) across face (dir, side); -1 at a wall. */
static long neighbour(const grid_t* G, int ex, int ey, int ez, int dir, int side)
{
    int c[3] = {ex, ey, ez};
    c[dir] += side;
    if (c[dir] < 0 || c[dir] >= G->ne[dir]) {
        if (!G->periodic[dir]) return -1;
        c[dir] = (c[dir] + G->ne[dir]) % G->ne[dir];
    }
    return c[0] + (long)G->ne[0] * (c[1] + (long)G->ne[1] * c[2]);
}

/* ======================================================================== */
/* Thermodynamics (Sect. 2.5-2.7)                                            */
/* ======================================================================== */

/* Saturation vapour pressure over liquid: Clausius-Clapeyron integrated with
 * constant heat capacities, L_v(T) = L_v0 + (c_pv - c_pl)(T - T_0). */
double cmref_pvsat(double T)
{
    double dc = CPV - CPL;
    return PTRIPLE * pow(T / TREF0, dc / RV) * exp((LV0 - dc * TREF0) / RV * (1.0 / TREF0 - 1.0 / T));
}

/* Ice (Sect. 2.5, Table 1): c_vi and L_f0, I_i0 = L_f0.  The paper
 * apportions the condensate "according to temperature" without stating
 * how; reading: liquid fraction 1 at and above the freezing point, 0 at and
 * below the homogeneous-nucleation temperature, linear in between. */
static const double CVI = 2100.0, LF0 = 0.3336e6;
static const double T_FREEZE = 273.15, T_ICENUC = 233.0;

/* Saturation vapour pressure over ice, Clausius-Clapeyron with constant
 * heat capacities: L_s(T) = L_v0 + L_f0 + (c_pv - c_vi)(T - T_0); equal to
 * the liquid one at the triple point T_0. */
double cmref_pvsat_ice(double T)
{
    double dc = CPV - CVI;
    return PTRIPLE * pow(T / TREF0, dc / RV) * exp((LV0 + LF0 - dc * TREF0) / RV * (1.0 / TREF0 - 1.0 / T));
}

double cmref_liquid_fraction(double T)
{
    if (T >= T_FREEZE) return 1.0;
    if (T <= T_ICENUC) return 0.0;
    return (T - T_ICENUC) / (T_FREEZE - T_ICENUC);
}

/* saturation specific humidity over the condensate mix at T: the vapour
 * pressure weighted by the liquid fraction (liquid only without ice) */
static double qvsat(double T, double rho, int ice)
{
    double pv = cmref_pvsat(T);
    if (ice) {
        double lam = cmref_liquid_fraction(T);
        pv = lam * pv + (1.0 - lam) * cmref_pvsat_ice(T);
    }
    return pv / (rho * RV * T);
}

/* Equilibrium internal energy I*(T; rho, q_t) (eq. total_internal_energy):
 * vapour at saturation (or all of q_t), the rest condensed, split between
 * liquid and ice by the liquid fraction (all liquid without ice). */
static double Istar(double T, double rho, double qt, int ice)
{
    double qv = qvsat(T, rho, ice);
    if (qv > qt) qv = qt;
    double qc = qt - qv;
    double lam = ice ? cmref_liquid_fraction(T) : 1.0;
    double ql = lam * qc, qi = qc - ql;
    return (1.0 - qt) * CVD * (T - TREF0) + qv * (CVV * (T - TREF0) + IV0) + ql * CVL * (T - TREF0) +
           qi * (CVI * (T - TREF0) - LF0);
}

/* Saturation adjustment: the root T of I*(T) - I = 0.  The oracle brackets
 * it and bisects to adjacent doubles (a different algorithm from the GPU's
 * Newton iteration, converging to the same root).  ql and qi at the root. */
void cmref_saturation_adjust_phase(double rho, double qt, double I, int ice, double* T_out, double* ql_out,
                                   double* qi_out)
{
    double Tu = TREF0 + (I - qt * IV0) / ((1.0 - qt) * CVD + qt * CVV);
    if (qt <= qvsat(Tu, rho, ice)) { *T_out = Tu; *ql_out = 0.0; *qi_out = 0.0; return; }
    double step = (LV0 + (ice ? LF0 : 0.0)) * qt / CVD;
    double lo = Tu, hi = Tu + step;
    while (Istar(hi, rho, qt, ice) - I < 0.0) hi += step;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (Istar(mid, rho, qt, ice) - I < 0.0) lo = mid; else hi = mid;
    }
    /* the two adjacent doubles bracket the root; take the one with the
     * smaller residual */
    double rl = fabs(Istar(lo, rho, qt, ice) - I), rh = fabs(Istar(hi, rho, qt, ice) - I);
    double T = (rl <= rh) ? lo : hi;
    double qv = qvsat(T, rho, ice);
    if (qv > qt) qv = qt;
    double lam = ice ? cmref_liquid_fraction(T) : 1.0;
    *T_out = T; *ql_out = lam * (qt - qv); *qi_out = (qt - qv) - *ql_out;
}

/* liquid-only adjustment (the model without ice) */
void cmref_saturation_adjust(double rho, double qt, double I, double* T_out, double* ql_out)
{
    double qi;
    cmref_saturation_adjust_phase(rho, qt, I, 0, T_out, ql_out, &qi);
}

typedef struct {
    double rho, u[3], e, qt;
    double T, p, c, h, thv, ql, qi, qv, Rm;
} prim_t;

/* State -> primitive/thermodynamic quantities at one node (z = height). */
static void thermo(const double* Yn, int nvar, int ice, double z, double g, prim_t* P)
{
    double rho = Yn[0];
    P->rho = rho;
    for (int c = 0; c < 3; ++c) P->u[c] = Yn[1 + c] / rho;
    P->e = Yn[4] / rho;
    P->qt = (nvar > 5) ? Yn[5] / rho : 0.0;
    double ke = 0.5 * (P->u[0] * P->u[0] + P->u[1] * P->u[1] + P->u[2] * P->u[2]);
    double I = P->e - ke - g * z;
    double qt = P->qt, T, ql, qi;
    if (nvar > 5) cmref_saturation_adjust_phase(rho, qt, I, ice, &T, &ql, &qi);
    else { T = TREF0 + I / CVD; ql = 0.0; qi = 0.0; }
    double qv = qt - ql - qi;
    double Rm = RD * (1.0 - qt) + RV * qv;
    double p = rho * Rm * T;
    double cvm = (1.0 - qt) * CVD + qv * CVV + ql * CVL + qi * CVI;
    double gam = (cvm + Rm) / cvm;
    P->T = T; P->ql = ql; P->qi = qi; P->qv = qv; P->Rm = Rm; P->p = p;
    P->c = sqrt(gam * Rm * T);
    P->h = P->e + p / rho;
    P->thv = T * pow(P00 / p, RD / CPD) * Rm / RD;
}

/* Per-node thermodynamic diagnostics for tests: T, p, q_l, theta_v. */
void cmref_thermo_nodes(int nvar, int ice, long n, const double* Y, const double* z, double g,
                        double* T, double* p, double* ql, double* thv)
{
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        double Yn[6];
        for (int v = 0; v < nvar; ++v) Yn[v] = Y[v * n + i];
        prim_t P; thermo(Yn, nvar, ice, z[i], g, &P);
        T[i] = P.T; p[i] = P.p; ql[i] = P.ql + P.qi; thv[i] = P.thv;
    }
}

/* ======================================================================== */
/* Fluxes                                                                   */
/* ======================================================================== */

/* Inviscid flux F1 (Sect. 3.1 compact form; momentum carries p - p_r). */
static void flux1(const prim_t* P, int nvar, double pr, double F[][3])
{
    for (int d = 0; d < 3; ++d) {
        double ud = P->u[d];
        F[0][d] = P->rho * ud;
        for (int c = 0; c < 3; ++c) F[1 + c][d] = P->rho * P->u[c] * ud + (c == d ? (P->p - pr) : 0.0);
        F[4][d] = (P->rho * P->e + P->p) * ud;
        if (nvar > 5) F[5][d] = P->rho * P->qt * ud;
    }
}

/* Rusanov numerical flux n.F1*: centred average plus half the maximum wave
 * speed times the jump (the factor 1/2 is the reading of the printed
 * formula, see the design notes). */
static void rusanov(const double* Ym, const prim_t* Pm, double prm,
                    const double* Yp, const prim_t* Pp, double prp,
                    const double n[3], int nvar, double* out)
{
    double Fm[6][3], Fp[6][3];
    flux1(Pm, nvar, prm, Fm);
    flux1(Pp, nvar, prp, Fp);
    double unm = Pm->u[0] * n[0] + Pm->u[1] * n[1] + Pm->u[2] * n[2];
    double unp = Pp->u[0] * n[0] + Pp->u[1] * n[1] + Pp->u[2] * n[2];
    double lm = fabs(unm) + Pm->c, lp = fabs(unp) + Pp->c;
    double lam = lm > lp ? lm : lp;
    for (int v = 0; v < nvar; ++v) {
        double fm = Fm[v][0] * n[0] + Fm[v][1] * n[1] + Fm[v][2] * n[2];
        double fp = Fp[v][0] * n[0] + Fp[v][1] * n[1] + Fp[v][2] * n[2];
        out[v] = 0.5 * (fm + fp) + 0.5 * lam * (Ym[v] - Yp[v]);
    }
}

/* Roe numerical flux (Sect. 3.1; Roe 1981) for dry air: centred average
 * minus half of sum_k |lambda_k| alpha_k r_k over the acoustic, entropy and
 * shear waves of the Roe-averaged state (weights sqrt(rho)).  With the
 * internal energy counted from T_0 (I = c_vd (T - T_0)), rho e_tot + rho
 * c_vd T_0 is the ideal-gas total energy whose Roe matrix is the textbook
 * one; the energy row here is that one minus c_vd T_0 times the mass row.
 * phi = g z at the face node (the same on both sides).  The momentum flux
 * carries p - p_r (p_r is continuous at the node, so only the centred part
 * sees it). */
static void roe(const prim_t* Pm, double prm, const prim_t* Pp, double prp, double phi, const double n[3],
                double* out)
{
    double Fm[6][3], Fp[6][3];
    flux1(Pm, 5, prm, Fm);
    flux1(Pp, 5, prp, Fp);
    double sm = sqrt(Pm->rho), sp = sqrt(Pp->rho);
    double wm = sm / (sm + sp), wp = sp / (sm + sp);
    double rh = sm * sp;
    double uh[3], du[3];
    for (int c = 0; c < 3; ++c) { uh[c] = wm * Pm->u[c] + wp * Pp->u[c]; du[c] = Pp->u[c] - Pm->u[c]; }
    double Hh = wm * Pm->h + wp * Pp->h;
    double q2 = uh[0] * uh[0] + uh[1] * uh[1] + uh[2] * uh[2];
    double c2 = (CPD / CVD - 1.0) * (Hh + CVD * TREF0 - 0.5 * q2 - phi);
    double ch = sqrt(c2);
    double unh = uh[0] * n[0] + uh[1] * n[1] + uh[2] * n[2];
    double dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
    double drho = Pp->rho - Pm->rho, dp = Pp->p - Pm->p;
    double a1 = (dp - rh * ch * dun) / (2.0 * c2);
    double a2 = drho - dp / c2;
    double a3 = (dp + rh * ch * dun) / (2.0 * c2);
    double l1 = fabs(unh - ch), l2 = fabs(unh), l3 = fabs(unh + ch);
    double D[5];
    D[0] = l1 * a1 + l2 * a2 + l3 * a3;
    double udu_t = uh[0] * du[0] + uh[1] * du[1] + uh[2] * du[2] - unh * dun;
    for (int c = 0; c < 3; ++c)
        D[1 + c] = l1 * a1 * (uh[c] - ch * n[c]) + l2 * a2 * uh[c] + l3 * a3 * (uh[c] + ch * n[c]) +
                   l2 * rh * (du[c] - dun * n[c]);
    D[4] = l1 * a1 * (Hh - ch * unh) + l2 * a2 * (0.5 * q2 + phi - CVD * TREF0) + l3 * a3 * (Hh + ch * unh) +
           l2 * rh * udu_t;
    for (int v = 0; v < 5; ++v) {
        double fm = Fm[v][0] * n[0] + Fm[v][1] * n[1] + Fm[v][2] * n[2];
        double fp = Fp[v][0] * n[0] + Fp[v][1] * n[1] + Fp[v][2] * n[2];
        out[v] = 0.5 * (fm + fp) - 0.5 * D[v];
    }
}

/* HLLC numerical flux (Sect. 3.1; Toro, Spruce & Speares 1994) for dry air,
 * with the wave-speed bounds of Davis, S_L = min(u_n - c) and S_R =
 * max(u_n + c) over both sides, the contact speed S* from the jump
 * conditions, and the star states rho_K (S_K - u_nK)/(S_K - S*) (1, u_K +
 * (S* - u_nK) n, e_K + (S* - u_nK)(S* + p_K / (rho_K (S_K - u_nK)))).  The
 * energy flux (rho e_tot + p) u_n is the form the jump conditions take
 * with any energy origin; the momentum flux carries p - p_r. */
static void hllc(const double* Ym, const prim_t* Pm, double prm, const double* Yp, const prim_t* Pp, double prp,
                 const double n[3], double* out)
{
    double Fm[6][3], Fp[6][3];
    flux1(Pm, 5, prm, Fm);
    flux1(Pp, 5, prp, Fp);
    double fm[5], fp[5];
    for (int v = 0; v < 5; ++v) {
        fm[v] = Fm[v][0] * n[0] + Fm[v][1] * n[1] + Fm[v][2] * n[2];
        fp[v] = Fp[v][0] * n[0] + Fp[v][1] * n[1] + Fp[v][2] * n[2];
    }
    double unm = Pm->u[0] * n[0] + Pm->u[1] * n[1] + Pm->u[2] * n[2];
    double unp = Pp->u[0] * n[0] + Pp->u[1] * n[1] + Pp->u[2] * n[2];
    double SL = fmin(unm - Pm->c, unp - Pp->c);
    double SR = fmax(unm + Pm->c, unp + Pp->c);
    if (SL >= 0.0) { for (int v = 0; v < 5; ++v) out[v] = fm[v]; return; }
    if (SR <= 0.0) { for (int v = 0; v < 5; ++v) out[v] = fp[v]; return; }
    double Ss = (Pp->p - Pm->p + Pm->rho * unm * (SL - unm) - Pp->rho * unp * (SR - unp)) /
                (Pm->rho * (SL - unm) - Pp->rho * (SR - unp));
    const prim_t* P = Ss >= 0.0 ? Pm : Pp;
    const double* Y = Ss >= 0.0 ? Ym : Yp;
    const double* f = Ss >= 0.0 ? fm : fp;
    double S = Ss >= 0.0 ? SL : SR, un = Ss >= 0.0 ? unm : unp;
    double fac = P->rho * (S - un) / (S - Ss);
    double Us[5];
    Us[0] = fac;
    for (int c = 0; c < 3; ++c) Us[1 + c] = fac * (P->u[c] + (Ss - un) * n[c]);
    Us[4] = fac * (P->e + (Ss - un) * (Ss + P->p / (P->rho * (S - un))));
    for (int v = 0; v < 5; ++v) out[v] = f[v] + S * (Us[v] - Y[v]);
}

/* the model's numerical flux: 0 Rusanov, 1 Roe, 2 HLLC */
static void numflux(int kind, const double* Ym, const prim_t* Pm, double prm, const double* Yp, const prim_t* Pp,
                    double prp, double phi, const double n[3], int nvar, double* out)
{
    if (kind == 1) roe(Pm, prm, Pp, prp, phi, n, out);
    else if (kind == 2) hllc(Ym, Pm, prm, Yp, Pp, prp, n, out);
    else rusanov(Ym, Pm, prm, Yp, Pp, prp, n, nvar, out);
}

/* Point evaluation of the Rusanov flux for the identity tests. */
void cmref_rusanov_point(int nvar, const double* Ym, const double* Yp, double zm, double zp,
                         double g, double prm, double prp, const double* n, double* out)
{
    prim_t Pm, Pp;
    thermo(Ym, nvar, 0, zm, g, &Pm);
    thermo(Yp, nvar, 0, zp, g, &Pp);
    rusanov(Ym, &Pm, prm, Yp, &Pp, prp, n, nvar, out);
}

/* Point evaluation of any of the numerical fluxes (dry for Roe and HLLC)
 * at a face node at height z, for the flux tests. */
void cmref_numflux_point(int kind, int nvar, const double* Ym, const double* Yp, double z, double g, double pr,
                         const double* n, double* out)
{
    prim_t Pm, Pp;
    thermo(Ym, nvar, 0, z, g, &Pm);
    thermo(Yp, nvar, 0, z, g, &Pp);
    numflux(kind, Ym, &Pm, pr, Yp, &Pp, pr, g * z, n, nvar, out);
}

/* ======================================================================== */
/* Model                                                                    */
/* ======================================================================== */
typedef struct {
    grid_t* G;
    cmref_model_desc m;
    double* pr;    /* reference pressure per node */
    double* rhor;  /* reference density per node */
    double* Yref;  /* the background state itself [nvar][nn] (zeros without one) */
    double Delta;  /* filter width (dx dy dz)^(1/3), dx = h/N */
    /* learned closure parameters (FP64 copy), optional */
    double* mlp;
    double* mlp_bf16;   /* bf16-rounded weights when the BF16 emulation is on */
    int mlp_n;
    double mlp_lo[12], mlp_hi[12];
    int mlp_use_fallback;
    long mlp_fallbacks;
} model_t;

void* cmref_model_create(void* grid, const cmref_model_desc* m, const double* Yref)
{
    if (m->flux < 0 || m->flux > 2 || (m->flux != 0 && m->nvar > 5)) return NULL;
    model_t* M = (model_t*)calloc(1, sizeof(model_t));
    M->G = (grid_t*)grid;
    M->m = *m;
    long nn = M->G->nnodes;
    M->pr = (double*)calloc(nn, sizeof(double));
    M->rhor = (double*)calloc(nn, sizeof(double));
    M->Yref = (double*)calloc((size_t)m->nvar * nn, sizeof(double));
    if (Yref) memcpy(M->Yref, Yref, sizeof(double) * (size_t)m->nvar * nn);
    if (Yref) {
        /* reference state: the unperturbed background pushed through the
         * same thermodynamic functions as the prognostic state */
        const double* z = M->G->xyz + 2 * nn;
        #pragma omp parallel for schedule(static)
        for (long i = 0; i < nn; ++i) {
            double Yn[6];
            for (int v = 0; v < m->nvar; ++v) Yn[v] = Yref[v * nn + i];
            prim_t P; thermo(Yn, m->nvar, m->ice, z[i], m->g, &P);
            M->pr[i] = P.p; M->rhor[i] = P.rho;
        }
    }
    grid_t* G = M->G;
    M->Delta = cbrt((G->h[0] / G->N) * (G->h[1] / G->N) * (G->h[2] / G->N));
    return M;
}

void cmref_model_destroy(void* h)
{
    model_t* M = (model_t*)h;
    if (!M) return;
    free(M->pr); free(M->rhor); free(M->Yref); free(M->mlp); free(M->mlp_bf16);
    free(M);
}

/* Exponential modal filter (Sect. 5.4, eq. exponential_filter), in place:
 * in every element, the deviation of each variable in mask (bit v) from the
 * background is expanded in Legendre modes along each direction, mode n
 * scaled by sigma(n) = exp(-alpha ((n - Nc)/(N - Nc))^order) for n > Nc (1
 * otherwise), and the background added back.  The 1-D filter is V diag(sigma)
 * V^-1 with V[i][n] = P_n(xi_i); the 3-D one, their Kronecker product, is
 * applied as a dense (N+1)^3 x (N+1)^3 matrix. */
void cmref_exp_filter(void* h, double* Y, int mask, int order, double alpha, int Nc)
{
    model_t* M = (model_t*)h;
    const grid_t* G = M->G;
    const int N = G->N, Q = N + 1, Np = Q * Q * Q;
    const long nn = G->nnodes;
    double V[CMREF_MAXQ][CMREF_MAXQ], A[CMREF_MAXQ][2 * CMREF_MAXQ], F1[CMREF_MAXQ][CMREF_MAXQ];
    for (int i = 0; i < Q; ++i)
        for (int n = 0; n < Q; ++n) {
            double P, dP;
            legendre(n, G->xi[i], &P, &dP);
            V[i][n] = P;
        }
    /* V^-1 by Gauss-Jordan elimination with partial pivoting on [V | I] */
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < 2 * Q; ++j) A[i][j] = j < Q ? V[i][j] : (j - Q == i ? 1.0 : 0.0);
    for (int c = 0; c < Q; ++c) {
        int piv = c;
        for (int r = c + 1; r < Q; ++r) if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        for (int j = 0; j < 2 * Q; ++j) { double t = A[c][j]; A[c][j] = A[piv][j]; A[piv][j] = t; }
        double d = A[c][c];
        for (int j = 0; j < 2 * Q; ++j) A[c][j] /= d;
        for (int r = 0; r < Q; ++r) {
            if (r == c) continue;
            double f = A[r][c];
            for (int j = 0; j < 2 * Q; ++j) A[r][j] -= f * A[c][j];
        }
    }
    double sig[CMREF_MAXQ];
    for (int n = 0; n < Q; ++n)
        sig[n] = n <= Nc ? 1.0 : exp(-alpha * pow((double)(n - Nc) / (double)(N - Nc), (double)order));
    for (int i = 0; i < Q; ++i)
        for (int l = 0; l < Q; ++l) {
            double acc = 0.0;
            for (int n = 0; n < Q; ++n) acc += V[i][n] * sig[n] * A[n][Q + l];
            F1[i][l] = acc;
        }
    double* F3 = (double*)malloc(sizeof(double) * Np * Np);
    for (int a = 0; a < Np; ++a) {
        int i = a % Q, j = (a / Q) % Q, k = a / (Q * Q);
        for (int b = 0; b < Np; ++b) {
            int l = b % Q, m = (b / Q) % Q, o = b / (Q * Q);
            F3[a * Np + b] = F1[i][l] * F1[j][m] * F1[k][o];
        }
    }
    const long ne = nn / Np;
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < ne; ++e) {
        double d[CMREF_MAXQ * CMREF_MAXQ * CMREF_MAXQ];
        for (int v = 0; v < M->m.nvar; ++v) {
            if (!(mask & (1 << v))) continue;
            double* y = Y + v * nn + e * Np;
            const double* yr = M->Yref + v * nn + e * Np;
            for (int b = 0; b < Np; ++b) d[b] = y[b] - yr[b];
            for (int a = 0; a < Np; ++a) {
                double acc = 0.0;
                for (int b = 0; b < Np; ++b) acc += F3[a * Np + b] * d[b];
                y[a] = yr[a] + acc;
            }
        }
    }
    free(F3);
}

void cmref_model_reference(void* h, double* pr, double* rhor)
{
    model_t* M = (model_t*)h;
    memcpy(pr, M->pr, sizeof(double) * M->G->nnodes);
    memcpy(rhor, M->rhor, sizeof(double) * M->G->nnodes);
}

/* learned closure hook, implemented in cmref_mlp.c */
int cmref_mlp_closure(const double* params, const double* Wb, const double* lo, const double* hi,
                      int use_fallback, const double gu[3][3], double N2, double Delta, double nu_sl,
                      double* nu, double* Prt);
void cmref_mlp_round_weights(const double* p, double* out);
int cmref_mlp_nparams(void);

/* params = [network, mean[12], std[12]]; bf16 != 0 evaluates the network
 * with bfloat16 matrix operands (the GPU's rounding points) */
void cmref_model_set_mlp(void* h, const double* params, int nparams,
                         const double* lo, const double* hi, int use_fallback, int bf16)
{
    model_t* M = (model_t*)h;
    free(M->mlp);
    free(M->mlp_bf16);
    M->mlp_bf16 = NULL;
    M->mlp = (double*)malloc(sizeof(double) * nparams);
    memcpy(M->mlp, params, sizeof(double) * nparams);
    if (bf16) {
        M->mlp_bf16 = (double*)malloc(sizeof(double) * cmref_mlp_nparams());
        cmref_mlp_round_weights(params, M->mlp_bf16);
    }
    M->mlp_n = nparams;
    memcpy(M->mlp_lo, lo, sizeof(double) * 12);
    memcpy(M->mlp_hi, hi, sizeof(double) * 12);
    M->mlp_use_fallback = use_fallback;
}

long cmref_model_mlp_fallbacks(void* h) { return ((model_t*)h)->mlp_fallbacks; }

/* Smagorinsky-Lilly eddy viscosity with the Richardson stability factor
 * (eq. smago and eq. richardson).  |S|^2 = 2 S_ij S_ij in both places. */
double cmref_smagorinsky(const double gu[3][3], double N2, double Cs, double Delta,
                         double Prt, int richardson)
{
    double SS = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double Sij = 0.5 * (gu[i][j] + gu[j][i]);
            SS += 2.0 * Sij * Sij;
        }
    if (SS <= 0.0) return 0.0;
    double fb = 1.0;
    if (richardson) {
        double Ri = N2 / SS;
        if (Ri > 0.0) {
            double a = 1.0 - Ri / Prt;
            fb = pow(a > 0.0 ? a : 0.0, 0.25);
        }
    }
    return (Cs * Delta) * (Cs * Delta) * sqrt(SS) * fb;
}

/* Vreman eddy viscosity (Sect. 4.2, eq. vreman-sgs): nu = 2.5 Cs^2
 * sqrt(B_beta / (u_ij u_ij)), beta_ij = sum_m Dm_m^2 u_i,m u_j,m, B_beta the
 * sum of the three principal 2x2 minors of beta; Dm the element size over N
 * per direction.  With richardson the same stability factor as
 * Smagorinsky-Lilly multiplies it (Ri = N^2 / |S|^2). */
double cmref_vreman(const double gu[3][3], double N2, double Cs, const double Dm[3], double Prt, int richardson)
{
    double aa = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) aa += gu[i][j] * gu[i][j];
    if (aa <= 0.0) return 0.0;
    double beta[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double b = 0.0;
            for (int m = 0; m < 3; ++m) b += Dm[m] * Dm[m] * gu[i][m] * gu[j][m];
            beta[i][j] = b;
        }
    double Bb = beta[0][0] * beta[1][1] + beta[0][0] * beta[2][2] + beta[1][1] * beta[2][2] -
                (beta[0][2] * beta[0][2] + beta[0][1] * beta[0][1] + beta[1][2] * beta[1][2]);
    if (Bb <= 0.0) return 0.0;
    double fb = 1.0;
    if (richardson) {
        double SS = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double Sij = 0.5 * (gu[i][j] + gu[j][i]);
                SS += 2.0 * Sij * Sij;
            }
        double Ri = SS > 0.0 ? N2 / SS : 0.0;
        if (Ri > 0.0) {
            double a = 1.0 - Ri / Prt;
            fb = pow(a > 0.0 ? a : 0.0, 0.25);
        }
    }
    return 2.5 * Cs * Cs * sqrt(Bb / aa) * fb;
}

void cmref_vreman_point(const double* gu9, double N2, double Cs, const double* Dm, double Prt, int richardson,
                        double* nu)
{
    double gu[3][3];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) gu[i][j] = gu9[3 * i + j];
    *nu = cmref_vreman(gu, N2, Cs, Dm, Prt, richardson);
}

void cmref_smagorinsky_point(const double* gu9, double N2, double Cs, double Delta, double Prt,
                             int richardson, double* nu)
{
    double gu[3][3];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) gu[i][j] = gu9[3 * i + j];
    *nu = cmref_smagorinsky(gu, N2, Cs, Delta, Prt, richardson);
}

/* Planted mistakes, for the tests that show that a pin fails when the
 * operator is wrong (0: none).  1: the diffusive flux doubled; 2: the sign
 * of tau flipped; 3: one-sided F2* (own side only); 4: the energy diffusion
 * -rho D_t grad h_tot dropped; 5: the d_qt (x) rho u momentum term dropped;
 * 6: the BR1 lift doubled. */
static int g_mutation = 0;
void cmref_set_mutation(int code) { g_mutation = code; }

/* gradient-variable slots */
enum { GU = 0, GV = 1, GW = 2, GH = 3 };

typedef struct {
    int nG;        /* number of gradient variables */
    int iq, ith;   /* slots of q_t and theta_v (-1 if absent) */
} gslots_t;

static gslots_t slots(const cmref_model_desc* m)
{
    gslots_t s; s.nG = 4; s.iq = -1; s.ith = -1;
    if (m->nvar > 5) s.iq = s.nG++;
    if (((m->closure == 2 || m->closure == 4) && m->richardson) || m->closure == 3) s.ith = s.nG++;
    return s;
}

/* workspace for one RHS evaluation */
typedef struct {
    prim_t* P;      /* per node */
    double* gvar;   /* [nG][nnodes] */
    double* grad;   /* [nG][3][nnodes] */
    double* F2;     /* [nvar][3][nnodes] */
} work_t;

/* BR1 auxiliary gradient of every gradient variable: chain-rule volume
 * derivative plus the lift of (g* - g^-) n with the centred g*; walls use
 * the interior value (g* = g^-). */
static void br1_gradients(const model_t* M, work_t* W, gslots_t s)
{
    const grid_t* G = M->G;
    int Q = G->Q, Np = G->Np, N = G->N; long nn = G->nnodes;
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < G->nelem; ++e) {
        int ex = (int)(e % G->ne[0]);
        int ey = (int)((e / G->ne[0]) % G->ne[1]);
        int ez = (int)(e / ((long)G->ne[0] * G->ne[1]));
        for (int k = 0; k < Q; ++k) for (int j = 0; j < Q; ++j) for (int i = 0; i < Q; ++i) {
            int loc = i + Q * (j + Q * k);
            long n = e * Np + loc;
            double J = G->J[n];
            for (int q = 0; q < s.nG; ++q) {
                const double* ge = W->gvar + q * nn + e * Np;
                double gr[3] = {0, 0, 0};
                for (int dir = 0; dir < 3; ++dir) {
                    double dg = dref(G, ge, dir, i, j, k);
                    for (int c = 0; c < 3; ++c) gr[c] += G->Ja[(3 * dir + c) * nn + n] / J * dg;
                }
                /* face lifts */
                int idx[3] = {i, j, k};
                for (int dir = 0; dir < 3; ++dir) {
                    for (int side = -1; side <= 1; side += 2) {
                        if ((side < 0 && idx[dir] != 0) || (side > 0 && idx[dir] != N)) continue;
                        long en = neighbour(G, ex, ey, ez, dir, side);
                        if (en < 0) continue; /* wall: g* = g^- */
                        int m3[3] = {i, j, k};
                        m3[dir] = (side < 0) ? N : 0;
                        long np = en * Np + m3[0] + Q * (m3[1] + Q * m3[2]);
                        double gm = W->gvar[q * nn + n], gp = W->gvar[q * nn + np];
                        double Ja0 = G->Ja[(3 * dir + 0) * nn + n];
                        double Ja1 = G->Ja[(3 * dir + 1) * nn + n];
                        double Ja2 = G->Ja[(3 * dir + 2) * nn + n];
                        double Js = sqrt(Ja0 * Ja0 + Ja1 * Ja1 + Ja2 * Ja2);
                        double nv[3] = {side * Ja0 / Js, side * Ja1 / Js, side * Ja2 / Js};
                        double lift = Js / (J * G->w[N]);
                        double gstar = 0.5 * (gm + gp);
                        if (g_mutation == 6) lift *= 2.0;
                        for (int c = 0; c < 3; ++c) gr[c] += lift * (gstar - gm) * nv[c];
                    }
                }
                for (int c = 0; c < 3; ++c) W->grad[(q * 3 + c) * nn + n] = gr[c];
            }
        }
    }
}

/* Diffusive flux F2 from the closure (Sect. 4): rho tau = -2 rho nu_t S,
 * rho d_qt = -rho D_t grad q_t, energy u.(rho tau) - rho D_t grad h_tot,
 * momentum also carries d_qt (x) rho u. */
static void diffusive_flux(model_t* M, work_t* W, gslots_t s)
{
    const grid_t* G = M->G; long nn = G->nnodes;
    const cmref_model_desc* m = &M->m;
    long fallbacks = 0;
    #pragma omp parallel for schedule(static) reduction(+:fallbacks)
    for (long n = 0; n < nn; ++n) {
        const prim_t* P = &W->P[n];
        double gu[3][3];
        for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) gu[i][j] = W->grad[(i * 3 + j) * nn + n];
        double N2 = 0.0;
        if (s.ith >= 0) N2 = m->g / P->thv * W->grad[(s.ith * 3 + 2) * nn + n];
        double nu = 0.0, Prt = m->Prt;
        if (m->closure == 1) nu = m->nu;
        else if (m->closure == 2) nu = cmref_smagorinsky(gu, N2, m->Cs, M->Delta, m->Prt, m->richardson);
        else if (m->closure == 4) {
            const double Dm[3] = {G->h[0] / G->N, G->h[1] / G->N, G->h[2] / G->N};
            nu = cmref_vreman(gu, N2, m->Cs, Dm, m->Prt, m->richardson);
        } else if (m->closure == 3) {
            double nu_sl = cmref_smagorinsky(gu, N2, m->Cs, M->Delta, m->Prt, m->richardson);
            if (M->mlp) {
                double nn_, pp_;
                int fb = cmref_mlp_closure(M->mlp, M->mlp_bf16, M->mlp_lo, M->mlp_hi, M->mlp_use_fallback,
                                           (const double (*)[3])gu, N2, M->Delta, nu_sl, &nn_, &pp_);
                if (fb) { nu = nu_sl; Prt = m->Prt; fallbacks++; }
                else { nu = nn_; Prt = pp_; }
            } else nu = nu_sl;
        }
        double Dt = nu / Prt;
        double S[3][3], rt[3][3];
        for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) S[i][j] = 0.5 * (gu[i][j] + gu[j][i]);
        for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) rt[i][j] = -2.0 * P->rho * nu * S[i][j];
        if (g_mutation == 2)
            for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) rt[i][j] = -rt[i][j];
        double rd[3] = {0, 0, 0};
        if (m->nvar > 5)
            for (int j = 0; j < 3; ++j) rd[j] = -P->rho * Dt * W->grad[(s.iq * 3 + j) * nn + n];
        for (int j = 0; j < 3; ++j) {
            W->F2[(0 * 3 + j) * nn + n] = (m->nvar > 5) ? rd[j] : 0.0;
            for (int i = 0; i < 3; ++i)
                W->F2[((1 + i) * 3 + j) * nn + n] =
                    rt[i][j] + ((m->nvar > 5 && g_mutation != 5) ? rd[j] * P->u[i] : 0.0);
            double ue = P->u[0] * rt[0][j] + P->u[1] * rt[1][j] + P->u[2] * rt[2][j];
            W->F2[(4 * 3 + j) * nn + n] = ue - (g_mutation == 4 ? 0.0 : P->rho * Dt * W->grad[(GH * 3 + j) * nn + n]);
            if (m->nvar > 5) W->F2[(5 * 3 + j) * nn + n] = rd[j];
        }
        if (g_mutation == 1)
            for (int q = 0; q < 3 * m->nvar; ++q) W->F2[(long)q * nn + n] *= 2.0;
    }
    M->mlp_fallbacks = fallbacks;
}

static void work_alloc(const model_t* M, work_t* W, gslots_t s)
{
    long nn = M->G->nnodes;
    W->P = (prim_t*)malloc(sizeof(prim_t) * nn);
    W->gvar = (double*)malloc(sizeof(double) * s.nG * nn);
    W->grad = (double*)calloc((size_t)s.nG * 3 * nn, sizeof(double));
    W->F2 = (double*)calloc((size_t)M->m.nvar * 3 * nn, sizeof(double));
}

static void work_free(work_t* W) { free(W->P); free(W->gvar); free(W->grad); free(W->F2); }

/* primitives and gradient variables at every node */
static void prepare(const model_t* M, const double* Y, work_t* W, gslots_t s)
{
    const grid_t* G = M->G; long nn = G->nnodes; int nvar = M->m.nvar;
    const double* z = G->xyz + 2 * nn;
    #pragma omp parallel for schedule(static)
    for (long n = 0; n < nn; ++n) {
        double Yn[6];
        for (int v = 0; v < nvar; ++v) Yn[v] = Y[v * nn + n];
        thermo(Yn, nvar, M->m.ice, z[n], M->m.g, &W->P[n]);
        const prim_t* P = &W->P[n];
        W->gvar[GU * nn + n] = P->u[0];
        W->gvar[GV * nn + n] = P->u[1];
        W->gvar[GW * nn + n] = P->u[2];
        W->gvar[GH * nn + n] = P->h;
        if (s.iq >= 0) W->gvar[s.iq * nn + n] = P->qt;
        if (s.ith >= 0) W->gvar[s.ith * nn + n] = P->thv;
    }
}

/* The semi-discrete DG operator (eq. matrixProblem, strong form):
 *   dY/dt = -(1/J) sum_d D_d (J a^d . F) + S
 *           + sum_faces J^s/(J w_N) (n.F^- - n.F^*)
 * with F = F1 + F2, F1* Rusanov, F2* centred; walls use the reflecting ghost
 * state for F1* and a prescribed n.F2*. */
static void rhs_eval(model_t* M, const double* Y, double* R, work_t* W)
{
    const grid_t* G = M->G;
    const cmref_model_desc* m = &M->m;
    int Q = G->Q, Np = G->Np, N = G->N, nvar = m->nvar; long nn = G->nnodes;
    gslots_t s = slots(m);
    prepare(M, Y, W, s);
    if (m->closure != 0) {
        br1_gradients(M, W, s);
        diffusive_flux(M, W, s);
    }
    const double* z = G->xyz + 2 * nn;
    /* total flux contracted with the metric: G_v^d = J a^d . F_v, per node */
    double* Gf = (double*)malloc(sizeof(double) * nvar * 3 * nn);
    #pragma omp parallel for schedule(static)
    for (long n = 0; n < nn; ++n) {
        double F[6][3];
        flux1(&W->P[n], nvar, M->pr[n], F);
        for (int v = 0; v < nvar; ++v) for (int d = 0; d < 3; ++d) F[v][d] += W->F2[(v * 3 + d) * nn + n];
        for (int v = 0; v < nvar; ++v)
            for (int dir = 0; dir < 3; ++dir) {
                double sum = 0.0;
                for (int c = 0; c < 3; ++c) sum += G->Ja[(3 * dir + c) * nn + n] * F[v][c];
                Gf[(v * 3 + dir) * nn + n] = sum;
            }
    }
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < G->nelem; ++e) {
        int ex = (int)(e % G->ne[0]);
        int ey = (int)((e / G->ne[0]) % G->ne[1]);
        int ez = (int)(e / ((long)G->ne[0] * G->ne[1]));
        for (int k = 0; k < Q; ++k) for (int j = 0; j < Q; ++j) for (int i = 0; i < Q; ++i) {
            int loc = i + Q * (j + Q * k);
            long n = e * Np + loc;
            double J = G->J[n];
            const prim_t* Pm = &W->P[n];
            double Rn[6];
            /* volume: conservative strong-form divergence */
            for (int v = 0; v < nvar; ++v) {
                double div = 0.0;
                for (int dir = 0; dir < 3; ++dir)
                    div += dref(G, Gf + (v * 3 + dir) * nn + e * Np, dir, i, j, k);
                Rn[v] = -div / J;
            }
            /* own total flux */
            double Fm[6][3];
            flux1(Pm, nvar, M->pr[n], Fm);
            for (int v = 0; v < nvar; ++v) for (int d = 0; d < 3; ++d) Fm[v][d] += W->F2[(v * 3 + d) * nn + n];
            double Ym[6];
            for (int v = 0; v < nvar; ++v) Ym[v] = Y[v * nn + n];
            /* faces this node lies on */
            int idx[3] = {i, j, k};
            for (int dir = 0; dir < 3; ++dir) {
                for (int side = -1; side <= 1; side += 2) {
                    if ((side < 0 && idx[dir] != 0) || (side > 0 && idx[dir] != N)) continue;
                    double Ja0 = G->Ja[(3 * dir + 0) * nn + n];
                    double Ja1 = G->Ja[(3 * dir + 1) * nn + n];
                    double Ja2 = G->Ja[(3 * dir + 2) * nn + n];
                    double Js = sqrt(Ja0 * Ja0 + Ja1 * Ja1 + Ja2 * Ja2);
                    double nv[3] = {side * Ja0 / Js, side * Ja1 / Js, side * Ja2 / Js};
                    double lift = Js / (J * G->w[N]);
                    double fstar[6], f2star[6];
                    long en = neighbour(G, ex, ey, ez, dir, side);
                    if (en >= 0) {
                        int m3[3] = {i, j, k};
                        m3[dir] = (side < 0) ? N : 0;
                        long np = en * Np + m3[0] + Q * (m3[1] + Q * m3[2]);
                        double Yp[6];
                        for (int v = 0; v < nvar; ++v) Yp[v] = Y[v * nn + np];
                        numflux(m->flux, Ym, Pm, M->pr[n], Yp, &W->P[np], M->pr[np], m->g * z[n], nv, nvar, fstar);
                        for (int v = 0; v < nvar; ++v) {
                            double a = 0.0, b = 0.0;
                            for (int c = 0; c < 3; ++c) {
                                a += W->F2[(v * 3 + c) * nn + n] * nv[c];
                                b += W->F2[(v * 3 + c) * nn + np] * nv[c];
                            }
                            f2star[v] = g_mutation == 3 ? a : 0.5 * (a + b);
                        }
                    } else {
                        /* reflecting ghost: u+ = u- - 2 (n.u-) n, scalars mirrored */
                        double Yp[6];
                        for (int v = 0; v < nvar; ++v) Yp[v] = Ym[v];
                        double mn = Ym[1] * nv[0] + Ym[2] * nv[1] + Ym[3] * nv[2];
                        for (int c = 0; c < 3; ++c) Yp[1 + c] = Ym[1 + c] - 2.0 * mn * nv[c];
                        prim_t Pp; thermo(Yp, nvar, m->ice, z[n], m->g, &Pp);
                        numflux(m->flux, Ym, Pm, M->pr[n], Yp, &Pp, M->pr[n], m->g * z[n], nv, nvar, fstar);
                        for (int v = 0; v < nvar; ++v) f2star[v] = 0.0;
                        if (m->closure != 0 && m->sfc_flux && dir == 2 && side < 0) {
                            /* prescribed upward surface fluxes; outward normal is -z */
                            double qf = (nvar > 5) ? m->qt_flux : 0.0;
                            double up_e = Pm->rho * (CPD * m->theta_flux + LV0 * qf);
                            f2star[4] = -up_e;
                            if (nvar > 5) { f2star[0] = -Pm->rho * qf; f2star[5] = -Pm->rho * qf; }
                        }
                    }
                    for (int v = 0; v < nvar; ++v) {
                        double fm = Fm[v][0] * nv[0] + Fm[v][1] * nv[1] + Fm[v][2] * nv[2];
                        Rn[v] += lift * (fm - (fstar[v] + f2star[v]));
                    }
                }
            }
            /* sources */
            Rn[3] -= (Pm->rho - M->rhor[n]) * m->g;
            if (m->f_cor != 0.0) {
                Rn[1] += m->f_cor * (Ym[2] - Pm->rho * m->v_g);
                Rn[2] -= m->f_cor * (Ym[1] - Pm->rho * m->u_g);
            }
            if (m->sponge && z[n] > m->sp_zs) {
                double zeta = (z[n] - m->sp_zs) / (m->sp_ztop - m->sp_zs);
                double tau = m->sp_alpha * pow(sin(0.5 * M_PI * zeta), m->sp_gamma);
                for (int c = 0; c < 3; ++c) Rn[1 + c] -= tau * (Ym[1 + c] - Pm->rho * m->sp_u[c]);
            }
            if (m->subsidence && m->closure != 0) {
                double zz = z[n] < m->sub_ztop ? z[n] : m->sub_ztop;
                double ws = -m->sub_w0 * sin(M_PI * zz / m->sub_ztop);
                Rn[4] -= Pm->rho * ws * W->grad[(GH * 3 + 2) * nn + n];
                if (nvar > 5) Rn[5] -= Pm->rho * ws * W->grad[(s.iq * 3 + 2) * nn + n];
            }
            for (int v = 0; v < nvar; ++v) R[v * nn + n] = Rn[v];
        }
    }
    free(Gf);
}

void cmref_rhs(void* h, const double* Y, double* R, double t)
{
    (void)t;
    model_t* M = (model_t*)h;
    work_t W; work_alloc(M, &W, slots(&M->m));
    rhs_eval(M, Y, R, &W);
    work_free(&W);
}

/* BR1 gradients ([nG][3][nnodes]) and F2 ([nvar][3][nnodes]) of a state. */
int cmref_gradients(void* h, const double* Y, double* grad, double* F2)
{
    model_t* M = (model_t*)h;
    gslots_t s = slots(&M->m);
    work_t W; work_alloc(M, &W, s);
    prepare(M, Y, &W, s);
    br1_gradients(M, &W, s);
    diffusive_flux(M, &W, s);
    long nn = M->G->nnodes;
    if (grad) memcpy(grad, W.grad, sizeof(double) * s.nG * 3 * nn);
    if (F2) memcpy(F2, W.F2, sizeof(double) * M->m.nvar * 3 * nn);
    work_free(&W);
    return s.nG;
}

/* ======================================================================== */
/* LSRK54 (Carpenter & Kennedy 1994, five stages, fourth order, 2N storage) */
/* ======================================================================== */
static const double LSRK_A[5] = {
    0.0,
    -567301805773.0 / 1357537059087.0,
    -2404267990393.0 / 2016746695238.0,
    -3550918686646.0 / 2091501179385.0,
    -1275806237668.0 / 842570457699.0};
static const double LSRK_B[5] = {
    1432997174477.0 / 9575080441755.0,
    5161836677717.0 / 13612068292357.0,
    1720146321549.0 / 2090206949498.0,
    3134564353537.0 / 4481467310338.0,
    2277821191437.0 / 14882151754819.0};
static const double LSRK_C[5] = {
    0.0,
    1432997174477.0 / 9575080441755.0,
    2526269341429.0 / 6820363266100.0,
    2006345519317.0 / 3224310063776.0,
    2802321613138.0 / 2924317926251.0};

void cmref_lsrk54_coeffs(double* A, double* B, double* C)
{
    for (int s = 0; s < 5; ++s) { A[s] = LSRK_A[s]; B[s] = LSRK_B[s]; C[s] = LSRK_C[s]; }
}

/* LSRK144 (Niegemann, Diehl & Busch 2012: fourteen stages, fourth order,
 * 2N storage, stability region fitted to DG operators), the integrator of
 * the paper's isotropic runs (Sect. 3.2).  Coefficients as published, to
 * sixteen digits; C_s are the stage times. */
static const double LSRK144_A[14] = {
    0.0, -0.7188012108672410, -0.7785331173421570, -0.0053282796654044, -0.8552979934029281,
    -3.9564138245774565, -1.5780575380587385, -2.0837094552574054, -0.7483334182761610,
    -0.7032861106563359, 0.0013917096117681, -0.0932075369637460, -0.9514200470875948,
    -7.1151571693922548};
static const double LSRK144_B[14] = {
    0.0367762454319673, 0.3136296607553959, 0.1531848691869027, 0.0030097086818182, 0.3326293790646110,
    0.2440251405350864, 0.3718879239592277, 0.6204126221582444, 0.1524043173028741, 0.0760894927419266,
    0.0077604214040978, 0.0024647284755382, 0.0780348340049386, 5.5059777270269628};
static const double LSRK144_C[14] = {
    0.0, 0.0367762454319673, 0.1249685262725025, 0.2446177702277698, 0.2476149531070420,
    0.2969311120382472, 0.3978149645802642, 0.5270854589440328, 0.6981269994175695,
    0.8190890835352128, 0.8527059887098624, 0.8604711817462826, 0.8627060376969976,
    0.8734213127600976};

void cmref_lsrk144_coeffs(double* A, double* B, double* C)
{
    for (int s = 0; s < 14; ++s) { A[s] = LSRK144_A[s]; B[s] = LSRK144_B[s]; C[s] = LSRK144_C[s]; }
}

/* nsteps steps in place of a 2N-storage scheme with ns stages: for each
 * stage dQ = A_s dQ + dt R(Y); Y += B_s dQ. */
static void lsrk_run(model_t* M, int ns, const double* A, const double* B, double* Y, double* dQ, double dt,
                     int nsteps)
{
    long n = (long)M->m.nvar * M->G->nnodes;
    double* R = (double*)malloc(sizeof(double) * n);
    work_t W; work_alloc(M, &W, slots(&M->m));
    for (int step = 0; step < nsteps; ++step) {
        for (int s = 0; s < ns; ++s) {
            rhs_eval(M, Y, R, &W);
            #pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) {
                dQ[i] = A[s] * dQ[i] + dt * R[i];
                Y[i] = Y[i] + B[s] * dQ[i];
            }
        }
    }
    work_free(&W);
    free(R);
}

/* LSRK54 steps in place (t: model time of the first step; the sources do
 * not depend on it) */
void cmref_lsrk_steps(void* h, double* Y, double* dQ, double t, double dt, int nsteps)
{
    (void)t;
    lsrk_run((model_t*)h, 5, LSRK_A, LSRK_B, Y, dQ, dt, nsteps);
}

/* LSRK144 steps in place */
void cmref_lsrk144_steps(void* h, double* Y, double* dQ, double t, double dt, int nsteps)
{
    (void)t;
    lsrk_run((model_t*)h, 14, LSRK144_A, LSRK144_B, Y, dQ, dt, nsteps);
}

/* ======================================================================== */
/* 1-D IMEX (HEVI, Sect. 3.2): the vertical acoustic operator of the dry    */
/* equations linearised about the background, treated implicitly in an     */
/* additive Runge-Kutta step (ARK2 of Giraldo, Kelly & Constantinescu 2013) */
/* ======================================================================== */

/* The linear operator on deviations d = Y - Y_ref of the five dry variables
 * along one vertical node line (fixed element column ex, ey and node i, j):
 * vertical flux F = (m, 0, 0, p', h m) with m = (rho w)', p' = (R_d/c_vd) E'
 * + (R_d T_0 - (R_d/c_vd) g z) rho' (the dry pressure linearised at rest) and
 * h = (E_r + p_r)/rho_r; L d = -(2/h_z) D F + lift (n.F - n.F*) at the
 * element's vertical faces with n.F* = n (F^- + F^+)/2 + c_r (d^- - d^+)/2
 * for every variable (c_r the background's sound speed: the vertical part
 * of the Rusanov penalty, horizontal momenta included), walls by the
 * mirrored ghost (m^+ = -m^-), and the buoyancy -g rho' in the vertical
 * momentum row.  Line vectors are ordered [var][element layer][k]. */
static void hevi_line_apply(const model_t* M, int ex, int ey, int i, int j, const double* dl, double* out)
{
    const grid_t* G = M->G;
    const int Q = G->Q, N = G->N, nz = G->ne[2];
    const long nn = G->nnodes;
    const double g = M->m.g, a = RD / CVD, hz = G->h[2];
    const double* z = G->xyz + 2 * nn;
    const int L = nz * Q;
#define IDX(v, ez, k) ((v) * L + (ez) * Q + (k))
    for (int ez = 0; ez < nz; ++ez) {
        long e = ex + (long)G->ne[0] * (ey + (long)G->ne[1] * ez);
        double F[5][CMREF_MAXQ], c[CMREF_MAXQ];
        for (int k = 0; k < Q; ++k) {
            long n = e * G->Np + i + Q * (j + Q * k);
            double rr = M->Yref[n], Er = M->Yref[4 * nn + n], pr = M->pr[n];
            double b = RD * TREF0 - a * g * z[n];
            double h = (Er + pr) / rr;
            double rho = dl[IDX(0, ez, k)], m = dl[IDX(3, ez, k)], E = dl[IDX(4, ez, k)];
            F[0][k] = m;
            F[1][k] = 0.0;
            F[2][k] = 0.0;
            F[3][k] = a * E + b * rho;
            F[4][k] = h * m;
            c[k] = sqrt(CPD / CVD * pr / rr);
        }
        for (int k = 0; k < Q; ++k) {
            for (int v = 0; v < 5; ++v) {
                double s = 0.0;
                for (int l = 0; l < Q; ++l) s += G->D[k * Q + l] * F[v][l];
                out[IDX(v, ez, k)] = -(2.0 / hz) * s;
            }
            out[IDX(3, ez, k)] -= g * dl[IDX(0, ez, k)];
        }
        /* faces: k = 0 (n = -1) and k = N (n = +1) */
        const double lift = (2.0 / hz) / G->w[N];
        for (int side = -1; side <= 1; side += 2) {
            int k = side < 0 ? 0 : N;
            double nrm = side;
            double dm[5], Fm[5], dp[5], Fp[5], lam = c[k];
            for (int v = 0; v < 5; ++v) { dm[v] = dl[IDX(v, ez, k)]; Fm[v] = F[v][k]; }
            long en = neighbour(G, ex, ey, ez, 2, side);
            if (en >= 0) {
                int ezn = (int)(en / ((long)G->ne[0] * G->ne[1]));
                int kn = side < 0 ? N : 0;
                long np = en * G->Np + i + Q * (j + Q * kn);
                double rr = M->Yref[np], Er = M->Yref[4 * nn + np], pr = M->pr[np];
                double b = RD * TREF0 - a * g * z[np];
                double h = (Er + pr) / rr;
                for (int v = 0; v < 5; ++v) dp[v] = dl[IDX(v, ezn, kn)];
                Fp[0] = dp[3];
                Fp[1] = 0.0;
                Fp[2] = 0.0;
                Fp[3] = a * dp[4] + b * dp[0];
                Fp[4] = h * dp[3];
                double cp = sqrt(CPD / CVD * pr / rr);
                if (cp > lam) lam = cp;
            } else {
                for (int v = 0; v < 5; ++v) { dp[v] = dm[v]; Fp[v] = Fm[v]; }
                dp[3] = -dm[3];
                Fp[0] = -Fm[0];
                Fp[4] = -Fm[4];
            }
            for (int v = 0; v < 5; ++v) {
                double fstar = 0.5 * nrm * (Fm[v] + Fp[v]) + 0.5 * lam * (dm[v] - dp[v]);
                out[IDX(v, ez, k)] += lift * (nrm * Fm[v] - fstar);
            }
        }
    }
#undef IDX
}

static void line_gather(const model_t* M, int ex, int ey, int i, int j, const double* Y, int dev, double* dl)
{
    const grid_t* G = M->G;
    const int Q = G->Q, nz = G->ne[2];
    const long nn = G->nnodes;
    for (int v = 0; v < 5; ++v)
        for (int ez = 0; ez < nz; ++ez)
            for (int k = 0; k < Q; ++k) {
                long e = ex + (long)G->ne[0] * (ey + (long)G->ne[1] * ez);
                long n = e * G->Np + i + Q * (j + Q * k);
                dl[v * nz * Q + ez * Q + k] = Y[v * nn + n] - (dev ? M->Yref[v * nn + n] : 0.0);
            }
}

static void line_scatter(const model_t* M, int ex, int ey, int i, int j, const double* dl, double* Y, int add_ref)
{
    const grid_t* G = M->G;
    const int Q = G->Q, nz = G->ne[2];
    const long nn = G->nnodes;
    for (int v = 0; v < 5; ++v)
        for (int ez = 0; ez < nz; ++ez)
            for (int k = 0; k < Q; ++k) {
                long e = ex + (long)G->ne[0] * (ey + (long)G->ne[1] * ez);
                long n = e * G->Np + i + Q * (j + Q * k);
                Y[v * nn + n] = dl[v * nz * Q + ez * Q + k] + (add_ref ? M->Yref[v * nn + n] : 0.0);
            }
}

/* LY = L (Y - Y_ref) on every node */
static void hevi_apply(const model_t* M, const double* Y, double* LY)
{
    const grid_t* G = M->G;
    const int Q = G->Q;
    const long nn = G->nnodes;
    const int nline = 5 * G->ne[2] * Q;
    memset(LY, 0, sizeof(double) * (size_t)M->m.nvar * nn);
    #pragma omp parallel for collapse(2) schedule(static)
    for (int ey = 0; ey < G->ne[1]; ++ey)
        for (int ex = 0; ex < G->ne[0]; ++ex) {
            double* dl = (double*)malloc(sizeof(double) * nline * 2);
            double* ol = dl + nline;
            for (int j = 0; j < Q; ++j)
                for (int i = 0; i < Q; ++i) {
                    line_gather(M, ex, ey, i, j, Y, 1, dl);
                    hevi_line_apply(M, ex, ey, i, j, dl, ol);
                    line_scatter(M, ex, ey, i, j, ol, LY, 0);
                }
            free(dl);
        }
}

/* Y_out = Y_ref + x with (I - tau L) x = B - Y_ref on the vertical line
 * (ex, ey, i, j): the line matrix assembled column by column from the
 * operator and solved by Gaussian elimination with partial pivoting.  A
 * holds n (n + 1) doubles and u 2 n, n = 5 nz Q. */
static void hevi_solve_line(const model_t* M, double tau, int ex, int ey, int i, int j, const double* B,
                            double* Yout, double* A, double* u)
{
    const int n = 5 * M->G->ne[2] * M->G->Q;
    double* Lu = u + n;
    for (int col = 0; col < n; ++col) {
        for (int r = 0; r < n; ++r) u[r] = r == col ? 1.0 : 0.0;
        hevi_line_apply(M, ex, ey, i, j, u, Lu);
        for (int r = 0; r < n; ++r) A[(size_t)r * (n + 1) + col] = u[r] - tau * Lu[r];
    }
    line_gather(M, ex, ey, i, j, B, 1, u);
    for (int r = 0; r < n; ++r) A[(size_t)r * (n + 1) + n] = u[r];
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[(size_t)r * (n + 1) + c]) > fabs(A[(size_t)piv * (n + 1) + c])) piv = r;
        if (piv != c)
            for (int k = 0; k <= n; ++k) {
                double t = A[(size_t)c * (n + 1) + k];
                A[(size_t)c * (n + 1) + k] = A[(size_t)piv * (n + 1) + k];
                A[(size_t)piv * (n + 1) + k] = t;
            }
        for (int r = c + 1; r < n; ++r) {
            double f = A[(size_t)r * (n + 1) + c] / A[(size_t)c * (n + 1) + c];
            if (f == 0.0) continue;
            for (int k = c; k <= n; ++k) A[(size_t)r * (n + 1) + k] -= f * A[(size_t)c * (n + 1) + k];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double v = A[(size_t)r * (n + 1) + n];
        for (int k = r + 1; k < n; ++k) v -= A[(size_t)r * (n + 1) + k] * u[k];
        u[r] = v / A[(size_t)r * (n + 1) + r];
    }
    line_scatter(M, ex, ey, i, j, u, Yout, 1);
}

/* the same on every line */
static void hevi_solve(const model_t* M, double tau, const double* B, double* Yout)
{
    const grid_t* G = M->G;
    const int Q = G->Q;
    const int n = 5 * G->ne[2] * Q;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int ey = 0; ey < G->ne[1]; ++ey)
        for (int ex = 0; ex < G->ne[0]; ++ex) {
            double* A = (double*)malloc(sizeof(double) * (size_t)n * (n + 1));
            double* u = (double*)malloc(sizeof(double) * 2 * n);
            for (int j = 0; j < Q; ++j)
                for (int i = 0; i < Q; ++i) hevi_solve_line(M, tau, ex, ey, i, j, B, Yout, A, u);
            free(A);
            free(u);
        }
}

/* ARK2 (Giraldo, Kelly & Constantinescu 2013): gamma = 1 - 1/sqrt2, delta =
 * 1/(2 sqrt2), a32 = (3 + 2 sqrt2)/6; explicit rows (0), (2 gamma), (1 - a32,
 * a32); implicit rows (0), (gamma, gamma), (delta, delta, gamma); weights
 * (delta, delta, gamma), shared by both. */
void cmref_ark2_coeffs(double* AE, double* AI, double* b)
{
    const double gam = 1.0 - 1.0 / sqrt(2.0), del = 1.0 / (2.0 * sqrt(2.0)), a32 = (3.0 + 2.0 * sqrt(2.0)) / 6.0;
    double ae[9] = {0, 0, 0, 2 * gam, 0, 0, 1 - a32, a32, 0};
    double ai[9] = {0, 0, 0, gam, gam, 0, del, del, gam};
    for (int q = 0; q < 9; ++q) { AE[q] = ae[q]; AI[q] = ai[q]; }
    b[0] = del; b[1] = del; b[2] = gam;
}

/* nsteps HEVI steps in place: stages Y_s solve Y_s - dt a_ss L(Y_s - Y_ref) =
 * Y_n + dt sum_{r<s} (aE_sr E_r + aI_sr L_r), E = R(Y) - L(Y - Y_ref);
 * Y_{n+1} = Y_n + dt sum_s b_s (E_s + L_s).  Dry models on flat meshes. */
int cmref_hevi_steps(void* h, double* Y, double t, double dt, int nsteps)
{
    model_t* M = (model_t*)h;
    (void)t;
    if (M->m.nvar != 5) return 1;
    const long nn = M->G->nnodes, n = (long)M->m.nvar * nn;
    double AE[9], AI[9], b[3];
    cmref_ark2_coeffs(AE, AI, b);
    double* Ys = (double*)malloc(sizeof(double) * n);
    double* Bs = (double*)malloc(sizeof(double) * n);
    double* E = (double*)malloc(sizeof(double) * 3 * n);
    double* Lt = (double*)malloc(sizeof(double) * 3 * n);
    work_t W; work_alloc(M, &W, slots(&M->m));
    for (int step = 0; step < nsteps; ++step) {
        for (int s = 0; s < 3; ++s) {
            for (long q = 0; q < n; ++q) {
                double acc = Y[q];
                for (int r = 0; r < s; ++r) acc += dt * (AE[3 * s + r] * E[r * n + q] + AI[3 * s + r] * Lt[r * n + q]);
                Bs[q] = acc;
            }
            if (AI[3 * s + s] != 0.0) {
                memcpy(Ys, Bs, sizeof(double) * n);   /* variables outside the operator */
                hevi_solve(M, dt * AI[3 * s + s], Bs, Ys);
            } else {
                memcpy(Ys, Bs, sizeof(double) * n);
            }
            rhs_eval(M, Ys, E + s * n, &W);
            hevi_apply(M, Ys, Lt + s * n);
            for (long q = 0; q < n; ++q) E[s * n + q] -= Lt[s * n + q];
        }
        for (long q = 0; q < n; ++q)
            Y[q] += dt * (b[0] * (E[q] + Lt[q]) + b[1] * (E[n + q] + Lt[n + q]) + b[2] * (E[2 * n + q] + Lt[2 * n + q]));
    }
    work_free(&W);
    free(Ys); free(Bs); free(E); free(Lt);
    return 0;
}

/* L (Y - Y_ref), for the operator's tests */
void cmref_hevi_operator(void* h, const double* Y, double* LY)
{
    hevi_apply((const model_t*)h, Y, LY);
}

/* the line solve on the listed lines only (line = (ex + ne0 ey) Q^2 + i +
 * Q j, each listed once), for checks at sizes where solving every line
 * would take minutes; Y must hold B beforehand, and the other lines keep it */
void cmref_hevi_solve_lines(void* h, double tau, const double* B, double* Y, const long* lines, int nl)
{
    const model_t* M = (const model_t*)h;
    const grid_t* G = M->G;
    const int Q = G->Q;
    const int n = 5 * G->ne[2] * Q;
    #pragma omp parallel for schedule(dynamic)
    for (int q = 0; q < nl; ++q) {
        const long line = lines[q];
        const long col = line / (Q * Q);
        const int node = (int)(line % (Q * Q));
        double* A = (double*)malloc(sizeof(double) * (size_t)n * (n + 1));
        double* u = (double*)malloc(sizeof(double) * 2 * n);
        hevi_solve_line(M, tau, (int)(col % G->ne[0]), (int)(col / G->ne[0]), node % Q, node / Q, B, Y, A, u);
        free(A);
        free(u);
    }
}

/* solve (I - tau L) x = B - Y_ref on every vertical line; returns Y_ref + x */
void cmref_hevi_solve(void* h, double tau, const double* B, double* Y)
{
    const model_t* M = (const model_t*)h;
    memcpy(Y, B, sizeof(double) * (size_t)M->m.nvar * M->G->nnodes);
    hevi_solve(M, tau, B, Y);
}

/* ======================================================================== */
/* Integrals (Sect. 6): sum of w_i w_j w_k |J| Y_v, Neumaier-compensated in  */
/* long double.  out[v] for v < nvar, then kinetic energy.                   */
/* ======================================================================== */
void cmref_integrals(void* h, const double* Y, double* out)
{
    model_t* M = (model_t*)h;
    grid_t* G = M->G; long nn = G->nnodes; int nvar = M->m.nvar;
    double* wJ = (double*)malloc(sizeof(double) * nn);
    cmref_grid_wJ(G, wJ);
    for (int v = 0; v <= nvar; ++v) {
        long double s = 0.0L, c = 0.0L;
        for (long n = 0; n < nn; ++n) {
            long double x;
            if (v < nvar) x = (long double)wJ[n] * Y[v * nn + n];
            else {
                double r = Y[n];
                double ke = 0.5 * (Y[nn + n] * Y[nn + n] + Y[2 * nn + n] * Y[2 * nn + n] + Y[3 * nn + n] * Y[3 * nn + n]) / r;
                x = (long double)wJ[n] * ke;
            }
            long double tt = s + x;
            if (fabsl(s) >= fabsl(x)) c += (s - tt) + x; else c += (x - tt) + s;
            s = tt;
        }
        out[v] = (double)(s + c);
    }
    free(wJ);
}

int cmref_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* thread count of the following parallel loops (timing on one thread) */
void cmref_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
