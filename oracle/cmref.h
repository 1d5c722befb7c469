/*
 * Oracle for the nodal discontinuous-Galerkin LES right-hand side and its
 * LSRK54 time step (Sridhar et al., "Large-eddy simulations with
 * ClimateMachine", GMD 2022, Sects. 2-4 and App. A).
 *
 * TEST INFRASTRUCTURE ONLY.  This plain, slow FP64 CPU implementation exists
 * to check the GPU library.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the GPU library.
 *
 * Layout of every state array: [var][element][node], node = i + Q*(j + Q*k)
 * with Q = N+1 (i along x), element = ex + ne0*(ey + ne1*ez).
 */
#ifndef CMREF_H
#define CMREF_H
#include <stdint.h>

#define CMREF_MAXQ 9

typedef struct {
    int N;              /* polynomial order */
    int ne[3];          /* elements per direction */
    double lo[3], hi[3];
    int periodic[3];
    int topo;           /* 0 flat, 1 Agnesi ridge z_sfc(x) */
    double topo_h, topo_a, topo_xc;
} cmref_grid_desc;

typedef struct {
    int nvar;           /* 5 dry (rho, rho u, rho v, rho w, rho e_tot), 6 moist (+ rho q_t) */
    int closure;        /* 0 none, 1 constant nu, 2 Smagorinsky-Lilly, 3 learned (MLP), 4 Vreman */
    double nu, Cs, Prt;
    int richardson;
    double g;
    double f_cor, u_g, v_g;
    int sponge;
    double sp_zs, sp_ztop, sp_alpha, sp_gamma, sp_u[3];
    int sfc_flux;
    double theta_flux, qt_flux;
    int subsidence;
    double sub_w0, sub_ztop;
    int flux;           /* inviscid numerical flux: 0 Rusanov, 1 Roe, 2 HLLC (the last two dry only) */
    int ice;            /* moist: condensate split between liquid and ice by temperature (else all liquid) */
} cmref_model_desc;

#endif
