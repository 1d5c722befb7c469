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
//   k_vsolve : (I - tau L) x = B - Y_ref on every vertical node line, 16
//              lanes per line: block-tridiagonal elimination over the
//              element layers with 15 x 15 blocks for (rho, rho w, rho e_tot)
//              (rows across lanes, partial pivoting by a DPP maximum and lane
//              permutes), 2 x 2 face systems for the horizontal momenta
//              (only the face penalty couples them); for backgrounds given
//              per node
//   k_vfactor, k_vapply4 / k_vapply, k_vmom: the same solve when every line
//              shares one matrix (background per level): the elimination
//              once per tau, then its application per line, and the momenta
//   k_href_table: the background's h_r and c_r per entry, for the solves
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
    double* scratch;           // solver workspace [n_lines][nz][60]
    double* hc;                // solver: h_r and c_r of every background entry [nref][2] (in the workspace)
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

// the solver's per-entry background table: h_r and c_r, each formed once
// per solve instead of at every node of every layer of every line
__global__ __launch_bounds__(256) void k_href_table(const HeviArgs A)
{
    const int64_t ri = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (ri >= A.nref) return;
    // the level of the entry only enters b, which the table does not hold
    const HRef r = href_at(A, ri, 0, 0);
    A.hc[2 * ri] = r.h;
    A.hc[2 * ri + 1] = r.c;
}

// background quantities of one node for the solver: h_r and c_r from the
// table, b from the node height (rho_r is not needed there)
__device__ __forceinline__ HRef href_tab(const HeviArgs& A, int64_t ri, int ez, int k)
{
    HRef r;
    r.rr = 0.0;
    r.h = A.hc[2 * ri];
    r.c = A.hc[2 * ri + 1];
    const double z = A.lo2 + ((double)ez + A.zg[k]) * A.h2;
    r.b = Phys::Rd * Phys::T0 - (Phys::Rd / Phys::cvd) * A.g * z;
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

constexpr int VS_N = 15;         // unknowns per element block: (rho, rho w, rho e_tot) x 5 nodes
constexpr int VS_LANES = 16;     // lanes per vertical line: lane r < 15 holds row r of the block
constexpr int VS_BLOCK = 64;     // one wave: four lines

// index of (variable 0 rho, 1 rho w, 2 rho e_tot; node k) in an element block
__device__ __forceinline__ int vb(int v3, int k) { return v3 * NQ + k; }

// one step of a maximum over the 16 lanes of a DPP row: the key of the
// partner lane given by the DPP control (0xB1: quad_perm [1,0,3,2]; 0x4E:
// quad_perm [2,3,0,1]; 0x141: row_half_mirror; 0x140: row_mirror; the four
// in this order pair every lane with every other of its row)
template <int CTRL>
__device__ __forceinline__ unsigned row_max_step(unsigned key)
{
    const unsigned o = (unsigned)__builtin_amdgcn_update_dpp((int)key, (int)key, CTRL, 0xF, 0xF, false);
    return o > key ? o : key;
}

// entry (row v, column w) of the Jacobian of the vertical flux
// (rho w, p', h rho w') w.r.t. (rho', m, E'):
//   [0 1 0; b 0 R_d/c_vd; 0 h 0]
// (w a compile-time column, v the lane's row: written out so that it is a
// select, not an indexed read of a register array)
__device__ __forceinline__ double jac_entry(const HRef& r, int v, int w)
{
    if (w == 0) return v == 1 ? r.b : 0.0;
    if (w == 1) return v == 0 ? 1.0 : (v == 2 ? r.h : 0.0);
    return v == 1 ? Phys::Rd / Phys::cvd : 0.0;
}

// row r = (v3, kr) of the layer block I - tau L_e on the vertical line of
// node (i, j) of element e (layer ez), and the row's coupling cpl to the
// nearest node of the neighbouring layer (bottom rows: the layer below, top
// rows: the layer above; zero at the walls).  Background from the table hc.
__device__ __forceinline__ void assemble_row(const HeviArgs& A, const double* sD, int e, int ez, int i, int j,
                                             int v3, int kr, double M[VS_N], double cpl[3])
{
    const double tau = A.tau, r2h = 2.0 / A.h2, lift = r2h * 10.0;
    const int nz = A.ne2;
    HRef rk[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) rk[k] = href_tab(A, href(A, e, ez, k, i + NQ * (j + NQ * k)), ez, k);
    const HRef ro = href_tab(A, href(A, e, ez, kr, i + NQ * (j + NQ * kr)), ez, kr);  // this row's node
    // the terms in this row's own node columns (w, kr) (the identity,
    // buoyancy, the face penalty or the wall) are summed first and enter
    // with a compare on the column's node, so that no entry is addressed by
    // a lane-dependent index
    double own[3];
#pragma unroll
    for (int w = 0; w < 3; ++w) own[w] = w == v3 ? 1.0 : 0.0;
    if (v3 == 1) own[0] += tau * A.g;
#pragma unroll
    for (int w = 0; w < 3; ++w) cpl[w] = 0.0;
    if (kr == 0 || kr == NQ - 1) {
        const int side = kr == 0 ? 0 : 1;
        const double nrm = side == 0 ? -1.0 : 1.0;
        const int ezn = ez + (side == 0 ? -1 : 1);
        if (ezn >= 0 && ezn < nz) {
            const int kn = NQ - 1 - kr;
            const int en = e + (side == 0 ? -A.ne01 : A.ne01);
            const HRef rn = href_tab(A, href(A, en, ezn, kn, i + NQ * (j + NQ * kn)), ezn, kn);
            const double lam = ro.c > rn.c ? ro.c : rn.c;
#pragma unroll
            for (int w = 0; w < 3; ++w) {
                own[w] -= tau * lift * (0.5 * nrm * jac_entry(ro, v3, w) - (v3 == w ? 0.5 * lam : 0.0));
                cpl[w] = -tau * lift * (-0.5 * nrm * jac_entry(rn, v3, w) + (v3 == w ? 0.5 * lam : 0.0));
            }
        } else {
            // wall: L_rho += lift n m, L_m -= lift c m, L_E += lift n h m
            if (v3 == 0) own[1] -= tau * lift * nrm;
            if (v3 == 1) own[1] += tau * lift * ro.c;
            if (v3 == 2) own[1] -= tau * lift * nrm * ro.h;
        }
    }
#pragma unroll
    for (int l = 0; l < NQ; ++l) {
        const double cf = tau * r2h * sD[kr * NQ + l];
#pragma unroll
        for (int w = 0; w < 3; ++w) M[vb(w, l)] = cf * jac_entry(rk[l], v3, w) + (l == kr ? own[w] : 0.0);
    }
}

// Y_out = Y_ref + x with (I - tau L) x = B - Y_ref on every vertical line
// (B and Y_out may be the same buffer: a line is read before it is written,
// and lines do not share nodes).
//
// Sixteen lanes per line, four lines per wave.  Over the element layers from
// the bottom, lane r assembles row r of the layer's 15 x 15 block I - tau L_e
// in registers, with the Schur update of its bottom-node rows by the layer
// below (the layers couple through one node pair, a rank-3 coupling); the
// block is solved by Gaussian elimination with partial pivoting across the
// lanes (the pivot by a DPP maximum over the row, the pivot row to the row's
// lanes by lane permutes; the lane that supplied the pivot for column c then
// owns unknown c) for the deviation and the three unit vectors at the top
// nodes.  Each layer leaves y_e and Z_e = W_e Btil_e in the workspace
// ([line][layer][60]) and its coupling to the next layer (S_e Btil_e, y_e at
// the top nodes) in LDS; the back substitution x_e = y_e - Z_e
// x_{e+1}(bottom nodes) runs from the top.  The horizontal
// momenta are coupled only by the face penalty: 2 x 2 systems per interior
// vertical face, solved by lanes 0-9.
template <typename R>
__global__ __launch_bounds__(VS_BLOCK) void k_vsolve(const HeviArgs A, const R* __restrict__ B, R* __restrict__ Yo,
                                                     int64_t n_lines)
{
    constexpr int NG = VS_BLOCK / VS_LANES;
    __shared__ double sQ[NG][24];         // per-layer broadcasts
    __shared__ double sG[NG][12];         // S_{e-1} Btil_{e-1} (9) and y_{e-1} at its top nodes (3)
    const int lane = threadIdx.x;
    const int gq = lane / VS_LANES, r = lane % VS_LANES;
    const int64_t line_id = (int64_t)blockIdx.x * NG + gq;
    const bool live = line_id < n_lines;                 // groups past the end compute, never write
    const int64_t line = live ? line_id : n_lines - 1;
    const bool rowl = r < VS_N;
    const int v3 = rowl ? r / NQ : 0, kr = rowl ? r % NQ : 0;
    const int node = (int)(line % (NQ * NQ));
    const int64_t col = line / (NQ * NQ);
    const int i = node % NQ, j = node / NQ;
    const int ex = (int)(col % A.ne0), ey = (int)(col / A.ne0);
    const double tau = A.tau, r2h = 2.0 / A.h2, lift = r2h * 10.0;
    const int nz = A.ne2;
    double* scr = A.scratch + line * (int64_t)nz * 60;   // [layer][60]: Z rows (45), then y (15)
    const int var = v3 == 0 ? 0 : (v3 == 1 ? 3 : 4);
    __shared__ double sD[NQ * NQ];  // the differentiation matrix (its row kr read per layer)
    if (lane < NQ * NQ) sD[lane] = A.D[lane];
    __syncthreads();
    for (int ez = 0; ez < nz; ++ez) {
        const int e = ex + A.ne0 * (ey + A.ne1 * ez);
        double M[VS_N], cpl[3];
        assemble_row(A, sD, e, ez, i, j, v3, kr, M, cpl);
        const int tnode = i + NQ * (j + NQ * kr);
        const int64_t ri = href(A, e, ez, kr, tnode);
        double b[4];
        b[0] = (double)B[var * A.nnS + (int64_t)e * SRUN + tnode] - sref<R>(A, var, ri);
        if (kr == 0 && ez > 0) {
            // Schur update of the bottom-node rows by the layers below
#pragma unroll
            for (int w = 0; w < 3; ++w) {
                double sg = 0.0;
#pragma unroll
                for (int q = 0; q < 3; ++q) sg += cpl[q] * sG[gq][3 * q + w];
                M[vb(w, 0)] -= sg;
            }
            double sy = 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) sy += cpl[q] * sG[gq][9 + q];
            b[0] -= sy;
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) b[1 + q] = r == vb(q, NQ - 1) ? 1.0 : 0.0;

        // elimination with partial pivoting across the lanes of the line;
        // the pivot row goes to the other lanes of the row by lane permutes
        bool used = !rowl;
        int mycol = -1;
        double myrp = 0.0;
        const int base = lane - r;  // first lane of this line's row
#pragma unroll
        for (int c = 0; c < VS_N; ++c) {
            // pivot: the largest |M[c]| among the rows not yet used, as one
            // 32-bit key per lane: the bits of |M[c]| in FP32 (their order is
            // the order of the magnitudes) with the low four replaced by
            // 15 - r, so the row maximum names its lane (the largest
            // magnitude to 2^-19, the lowest row among those); used rows 0
            unsigned key = used ? 0u : ((__float_as_uint((float)fabs(M[c])) & ~0xFu) | (unsigned)(15 - r));
            key = row_max_step<0xB1>(key);
            key = row_max_step<0x4E>(key);
            key = row_max_step<0x141>(key);
            key = row_max_step<0x140>(key);
            const int who = 15 - (int)(key & 0xFu);
            // the pivot row's entries right of c and its right-hand sides go
            // to the row's lanes one at a time; the rows not yet used subtract
            // their multiple of it (the multiplier is zero on the pivot row
            // and on used rows, which a finite pivot row leaves unchanged)
            const int src = base + who;
            // the pivot's reciprocal (Newton-refined hardware estimate; the
            // pivot of a nonsingular block is finite and nonzero) serves the
            // multipliers here and, kept by the pivot lane, its unknown in the
            // back substitution
            const double rp = frcp(__shfl(M[c], src));
            const double f = (!used && r != who) ? M[c] * rp : 0.0;
            if (r == who) {
                used = true;
                mycol = c;
                myrp = rp;
            }
#pragma unroll
            for (int q = c + 1; q < VS_N; ++q) M[q] = fma(-f, __shfl(M[q], src), M[q]);
#pragma unroll
            for (int q = 0; q < 4; ++q) b[q] = fma(-f, __shfl(b[q], src), b[q]);
        }
        // back substitution, column by column from the last: the owner of
        // unknown c finishes it, the others take it by a lane permute and
        // subtract
        double x[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = VS_N - 1; c >= 0; --c) {
            double xc[4];
            const bool mine = mycol == c;
#pragma unroll
            for (int q = 0; q < 4; ++q) x[q] = mine ? b[q] * myrp : x[q];
            // the lane of this row that owns unknown c
            const int own = __builtin_ctzll(__ballot(mycol == c) >> base);
#pragma unroll
            for (int q = 0; q < 4; ++q) xc[q] = __shfl(x[q], base + own);
            const double u = (mycol >= 0 && mycol < c) ? M[c] : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) b[q] = fma(-u, xc[q], b[q]);
        }
        // broadcasts: S_e (W at the top-node unknowns), y there, and Btil_e
        // (the coupling rows of the top nodes)
        if (mycol >= 0 && mycol % NQ == NQ - 1) {
            const int v = mycol / NQ;
#pragma unroll
            for (int q = 0; q < 3; ++q) sQ[gq][3 * v + q] = x[1 + q];
            sQ[gq][9 + v] = x[0];
        }
        if (rowl && kr == NQ - 1) {
#pragma unroll
            for (int w = 0; w < 3; ++w) sQ[gq][12 + 3 * v3 + w] = cpl[w];
        }
        __syncthreads();
        double Bt[3][3];
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int w = 0; w < 3; ++w) Bt[q][w] = sQ[gq][12 + 3 * q + w];
        // for the next layer's bottom rows (per line, in LDS): lane r < 9
        // forms entry r of S_e Btil_e, lanes 9-11 copy y_e
        if (r < 9) {
            const int v = r / 3, w = r % 3;
            double sg = 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) sg += sQ[gq][3 * v + q] * sQ[gq][12 + 3 * q + w];
            sG[gq][r] = sg;
        } else if (r < 12) {
            sG[gq][r] = sQ[gq][r];
        }
        if (mycol >= 0 && live) {
#pragma unroll
            for (int w = 0; w < 3; ++w) {
                double sz = 0.0;
#pragma unroll
                for (int q = 0; q < 3; ++q) sz += x[1 + q] * Bt[q][w];
                scr[ez * 60 + mycol * 3 + w] = sz;
            }
            scr[ez * 60 + 45 + mycol] = x[0];
        }
        __syncthreads();
    }
    // back substitution over the layers from the top: lane r takes unknown r
    double xb[3] = {0.0, 0.0, 0.0};
    for (int ez = nz - 1; ez >= 0; --ez) {
        const int e = ex + A.ne0 * (ey + A.ne1 * ez);
        double xr = 0.0;
        if (rowl) {
            xr = scr[ez * 60 + 45 + r];
            if (ez < nz - 1)
#pragma unroll
                for (int w = 0; w < 3; ++w) xr -= scr[ez * 60 + r * 3 + w] * xb[w];
            const int tnode = i + NQ * (j + NQ * kr);
            const int64_t ri = href(A, e, ez, kr, tnode);
            if (live) Yo[var * A.nnS + (int64_t)e * SRUN + tnode] = (R)(sref<R>(A, var, ri) + xr);
            if (kr == 0) sQ[gq][v3] = xr;
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < 3; ++w) xb[w] = sQ[gq][w];
        __syncthreads();
    }
    // horizontal momenta: identity except the 2 x 2 systems of the interior
    // vertical faces, [1 + s, -s; -s, 1 + s] with s = tau lift lam / 2; lane
    // r < 10 takes variable 1 + r / 5 at node r % 5 of every layer
    if (r < 2 * NQ && live) {
        const int v = 1 + r / NQ, k = r % NQ;
        for (int ez = 0; ez < nz; ++ez) {
            const int e = ex + A.ne0 * (ey + A.ne1 * ez);
            const int tnode = i + NQ * (j + NQ * k);
            const int64_t ri = href(A, e, ez, k, tnode);
            if (k == NQ - 1 && ez < nz - 1) {
                // the pair (top node of ez, bottom node of ez + 1)
                const int en = e + A.ne01;
                const int tn = i + NQ * j;
                const int64_t rin = href(A, en, ez + 1, 0, tn);
                const HRef ra = href_tab(A, ri, ez, k), rb = href_tab(A, rin, ez + 1, 0);
                const double lam = ra.c > rb.c ? ra.c : rb.c;
                const double sv = 0.5 * tau * lift * lam, al = 1.0 + sv, det = al * al - sv * sv;
                const double xa = (double)B[v * A.nnS + (int64_t)e * SRUN + tnode] - sref<R>(A, v, ri);
                const double xbv = (double)B[v * A.nnS + (int64_t)en * SRUN + tn] - sref<R>(A, v, rin);
                Yo[v * A.nnS + (int64_t)e * SRUN + tnode] = (R)(sref<R>(A, v, ri) + (al * xa + sv * xbv) / det);
                Yo[v * A.nnS + (int64_t)en * SRUN + tn] = (R)(sref<R>(A, v, rin) + (sv * xa + al * xbv) / det);
            } else if (!(k == 0 && ez > 0)) {
                Yo[v * A.nnS + (int64_t)e * SRUN + tnode] = B[v * A.nnS + (int64_t)e * SRUN + tnode];
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

// ---- lines with a common matrix ------------------------------------------
// With the background given per level (horizontally uniform) on a flat mesh,
// every vertical line has the same matrix I - tau L: only the right-hand
// sides differ.  The block elimination over the layers is then done once per
// tau (k_vfactor), and each line only applies it (k_vapply).  Per layer e the
// factor holds Minv_e, the inverse of the layer block after the Schur update
// of its bottom-node rows by the layers below; Z_e = W_e Btil_e (W_e: the
// columns of Minv_e at the top-node rows, Btil_e: the coupling rows of the
// top nodes to the layer above); and Cb_e, the coupling rows of the bottom
// nodes to the layer below: HEVI_FAC doubles per layer.
constexpr int HEVI_FAC = VS_N * VS_N + 3 * VS_N + 9;

// one block of 64 threads: the line of node (0, 0) of element column (0, 0);
// each layer's block inverted by Gauss-Jordan elimination with partial
// pivoting in LDS (the largest magnitude, the lowest row on ties)
__global__ __launch_bounds__(64) void k_vfactor(const HeviArgs A, double* __restrict__ F)
{
    __shared__ double T[VS_N][2 * VS_N];  // [block | identity] -> [I | Minv]
    __shared__ double sD[NQ * NQ];
    __shared__ double Gs[9];              // S_{e-1} Btil_{e-1}
    __shared__ double Ct[9], Cb[9];       // coupling rows of the top / bottom nodes
    __shared__ double prow[2 * VS_N], fcol[VS_N];
    __shared__ int piv;
    const int t = threadIdx.x;
    const int nz = A.ne2;
    if (t < NQ * NQ) sD[t] = A.D[t];
    if (t < 9) Gs[t] = 0.0;
    __syncthreads();
    for (int ez = 0; ez < nz; ++ez) {
        const int e = A.ne01 * ez;
        if (t < VS_N) {
            const int v3 = t / NQ, kr = t % NQ;
            double M[VS_N], cpl[3];
            assemble_row(A, sD, e, ez, 0, 0, v3, kr, M, cpl);
            if (kr == 0 && ez > 0) {
                for (int w = 0; w < 3; ++w) {
                    double sg = 0.0;
                    for (int q = 0; q < 3; ++q) sg += cpl[q] * Gs[3 * q + w];
                    M[vb(w, 0)] -= sg;
                }
            }
            for (int c = 0; c < VS_N; ++c) {
                T[t][c] = M[c];
                T[t][VS_N + c] = c == t ? 1.0 : 0.0;
            }
            if (kr == 0)
                for (int q = 0; q < 3; ++q) Cb[3 * v3 + q] = cpl[q];
            if (kr == NQ - 1)
                for (int q = 0; q < 3; ++q) Ct[3 * v3 + q] = cpl[q];
        }
        __syncthreads();
        for (int c = 0; c < VS_N; ++c) {
            if (t == 0) {
                int p = c;
                for (int r = c + 1; r < VS_N; ++r)
                    if (fabs(T[r][c]) > fabs(T[p][c])) p = r;
                piv = p;
            }
            __syncthreads();
            const int p = piv;
            if (p != c && t < 2 * VS_N) {
                const double a = T[c][t];
                T[c][t] = T[p][t];
                T[p][t] = a;
            }
            __syncthreads();
            if (t < 2 * VS_N) prow[t] = T[c][t] / T[c][c];
            if (t < VS_N) fcol[t] = T[t][c];
            __syncthreads();
            for (int q = t; q < VS_N * 2 * VS_N; q += 64) {
                const int r = q / (2 * VS_N), k = q % (2 * VS_N);
                T[r][k] = r == c ? prow[k] : T[r][k] - fcol[r] * prow[k];
            }
            __syncthreads();
        }
        // Minv, Z = W Btil with W = Minv(:, top rows), the coupling rows of
        // the bottom nodes, and G = S Btil for the next layer (S = W at the
        // top rows)
        double* Fe = F + (int64_t)ez * HEVI_FAC;
        for (int q = t; q < VS_N * VS_N; q += 64) Fe[q] = T[q / VS_N][VS_N + q % VS_N];
        if (t < 3 * VS_N) {
            const int r = t / 3, w = t % 3;
            double z = 0.0;
            for (int q = 0; q < 3; ++q) z += T[r][VS_N + vb(q, NQ - 1)] * Ct[3 * q + w];
            Fe[VS_N * VS_N + t] = z;
        }
        if (t < 9) Fe[VS_N * VS_N + 3 * VS_N + t] = Cb[t];
        __syncthreads();
        if (t < 9) {
            const int v = t / 3, w = t % 3;
            double g = 0.0;
            for (int q = 0; q < 3; ++q) g += T[vb(v, NQ - 1)][VS_N + vb(q, NQ - 1)] * Ct[3 * q + w];
            Gs[t] = g;
        }
        __syncthreads();
    }
}

// the line's 15 unknowns of layer ez (variables rho, rho w, rho e_tot at its
// five nodes) as deviations from the background
template <typename R>
__device__ __forceinline__ void load_layer(const HeviArgs& A, const R* B, int e, int ez, int i, int j, double b[VS_N])
{
#pragma unroll
    for (int r = 0; r < VS_N; ++r) {
        const int v3 = r / NQ, kr = r % NQ, var = v3 == 0 ? 0 : (v3 == 1 ? 3 : 4);
        const int tnode = i + NQ * (j + NQ * kr);
        b[r] = (double)B[var * A.nnS + (int64_t)e * SRUN + tnode] - sref<R>(A, var, href(A, e, ez, kr, tnode));
    }
}

// one thread per vertical line, 64 lines per block (one wave); each layer's
// factor is staged in LDS (two buffers: the next layer's copy is issued
// before the current layer's arithmetic) and read by every thread at the
// same address.  Forward over the layers y_e = Minv_e (b_e - Cb_e
// y_{e-1}(top nodes)), y_e kept in the workspace ([layer][row][line]); back
// substitution x_e = y_e - Z_e x_{e+1}(bottom nodes).  The next layer's
// state loads are also issued before the current layer's arithmetic.
// Threads past the last line compute on the last line and write nothing, so
// that every thread reaches the barriers.  B and Y may be the same buffer (a
// line is read before it is written, and lines do not share nodes).
template <typename R, bool WHOLE>
__global__ __launch_bounds__(64) void k_vapply(const HeviArgs A, const double* __restrict__ F, const R* B, R* Y,
                                               int64_t n_lines)
{
    // WHOLE: the factor of every layer in LDS at once, copied at entry (no
    // barrier per layer); else two layer buffers
    extern __shared__ double sFw[];
    __shared__ double sF[WHOLE ? 1 : 2][WHOLE ? 1 : HEVI_FAC];
    const int nz = A.ne2;
    const int t = threadIdx.x;
    const int64_t line_id = (int64_t)blockIdx.x * 64 + t;
    const bool live = line_id < n_lines;
    const int64_t line = live ? line_id : n_lines - 1;
    const int node = (int)(line % (NQ * NQ));
    const int64_t col = line / (NQ * NQ);
    const int i = node % NQ, j = node / NQ;
    const int ex = (int)(col % A.ne0), ey = (int)(col / A.ne0);
    double* ys = A.scratch;
    if (WHOLE)
        for (int q = t; q < nz * HEVI_FAC; q += 64) sFw[q] = F[q];
    else
        for (int q = t; q < HEVI_FAC; q += 64) sF[0][q] = F[q];
    double yprev[3] = {0.0, 0.0, 0.0};
    double bn[VS_N];
    load_layer<R>(A, B, ex + A.ne0 * ey, 0, i, j, bn);
    __syncthreads();
    for (int ez = 0; ez < nz; ++ez) {
        const double* Fe = WHOLE ? sFw + ez * HEVI_FAC : sF[ez & 1];
        if (!WHOLE && ez + 1 < nz)
            for (int q = t; q < HEVI_FAC; q += 64) sF[(ez + 1) & 1][q] = F[(int64_t)(ez + 1) * HEVI_FAC + q];
        double b[VS_N];
#pragma unroll
        for (int r = 0; r < VS_N; ++r) b[r] = bn[r];
        if (ez + 1 < nz) load_layer<R>(A, B, ex + A.ne0 * (ey + A.ne1 * (ez + 1)), ez + 1, i, j, bn);
#pragma unroll
        for (int w = 0; w < 3; ++w)
#pragma unroll
            for (int q = 0; q < 3; ++q) b[vb(w, 0)] -= Fe[VS_N * VS_N + 3 * VS_N + 3 * w + q] * yprev[q];
#pragma unroll
        for (int r = 0; r < VS_N; ++r) {
            double y = 0.0;
#pragma unroll
            for (int c = 0; c < VS_N; ++c) y += Fe[r * VS_N + c] * b[c];
            if (live) ys[((int64_t)ez * VS_N + r) * n_lines + line] = y;
            if (r % NQ == NQ - 1) yprev[r / NQ] = y;
        }
        if (!WHOLE) __syncthreads();
    }
    // the last layer's factor is still in its buffer
    double xb[3] = {0.0, 0.0, 0.0};
    double yn[VS_N];
#pragma unroll
    for (int r = 0; r < VS_N; ++r) yn[r] = ys[((int64_t)(nz - 1) * VS_N + r) * n_lines + line];
    for (int ez = nz - 1; ez >= 0; --ez) {
        const int e = ex + A.ne0 * (ey + A.ne1 * ez);
        const double* Fe = WHOLE ? sFw + ez * HEVI_FAC : sF[ez & 1];
        if (!WHOLE && ez > 0)
            for (int q = t; q < HEVI_FAC; q += 64) sF[(ez - 1) & 1][q] = F[(int64_t)(ez - 1) * HEVI_FAC + q];
        double x[VS_N];
#pragma unroll
        for (int r = 0; r < VS_N; ++r) x[r] = yn[r];
        if (ez > 0)
#pragma unroll
            for (int r = 0; r < VS_N; ++r) yn[r] = ys[((int64_t)(ez - 1) * VS_N + r) * n_lines + line];
#pragma unroll
        for (int r = 0; r < VS_N; ++r)
#pragma unroll
            for (int w = 0; w < 3; ++w) x[r] -= Fe[VS_N * VS_N + 3 * r + w] * xb[w];
        if (live) {
#pragma unroll
            for (int r = 0; r < VS_N; ++r) {
                const int v3 = r / NQ, kr = r % NQ, var = v3 == 0 ? 0 : (v3 == 1 ? 3 : 4);
                const int tnode = i + NQ * (j + NQ * kr);
                Y[var * A.nnS + (int64_t)e * SRUN + tnode] = (R)(sref<R>(A, var, href(A, e, ez, kr, tnode)) + x[r]);
            }
        }
#pragma unroll
        for (int w = 0; w < 3; ++w) xb[w] = x[vb(w, 0)];
        if (!WHOLE) __syncthreads();
    }
}

// a double from lane s of this lane's DPP quad
template <int S>
__device__ __forceinline__ double quad_bcast(double x)
{
    constexpr int CTRL = S | (S << 2) | (S << 4) | (S << 6);
    const unsigned long long bits = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)bits, (int)(unsigned)bits, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(bits >> 32), (int)(unsigned)(bits >> 32), CTRL, 0xF,
                                               0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// the same application with four lanes per line (a DPP quad, 16 lines per
// wave, 64 per 256-thread block), the factor of every layer in LDS: lane q
// holds rows q, q + 4, q + 8 (and q + 12 for q < 3) of the line's 15; the
// right-hand sides of the other lanes and the coupling values come by DPP
// quad broadcasts
template <typename R>
__global__ __launch_bounds__(256) void k_vapply4(const HeviArgs A, const double* __restrict__ F, const R* B, R* Y,
                                                 int64_t n_lines)
{
    extern __shared__ double sFw[];  // [nz][HEVI_FAC]
    const int nz = A.ne2;
    for (int q = threadIdx.x; q < nz * HEVI_FAC; q += 256) sFw[q] = F[q];
    __syncthreads();
    const int q = threadIdx.x & 3;
    const int64_t line_id = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 2;
    // every lane of a quad takes part in the broadcasts; lanes past the last
    // line compute on the last line and write nothing
    const bool live = line_id < n_lines;
    const int64_t line = live ? line_id : n_lines - 1;
    const int node = (int)(line % (NQ * NQ));
    const int64_t col = line / (NQ * NQ);
    const int i = node % NQ, j = node / NQ;
    const int ex = (int)(col % A.ne0), ey = (int)(col / A.ne0);
    double* ys = A.scratch;
    // this lane's rows r = q + 4 m (m = 3 only for q < 3)
    int var[4], tnode[4], kr[4];
    bool has[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int r = q + 4 * m;
        has[m] = r < VS_N;
        const int rr = has[m] ? r : 0, v3 = rr / NQ;
        kr[m] = rr % NQ;
        var[m] = v3 == 0 ? 0 : (v3 == 1 ? 3 : 4);
        tnode[m] = i + NQ * (j + NQ * kr[m]);
    }
    auto load = [&](int ez, double* b) {
        const int e = ex + A.ne0 * (ey + A.ne1 * ez);
#pragma unroll
        for (int m = 0; m < 4; ++m)
            b[m] = has[m] ? (double)B[var[m] * A.nnS + (int64_t)e * SRUN + tnode[m]] -
                                sref<R>(A, var[m], href(A, e, ez, kr[m], tnode[m]))
                          : 0.0;
    };
    double yprev[3] = {0.0, 0.0, 0.0};
    double bn[4];
    load(0, bn);
    for (int ez = 0; ez < nz; ++ez) {
        const double* Fe = sFw + ez * HEVI_FAC;
        double bm[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) bm[m] = bn[m];
        if (ez + 1 < nz) load(ez + 1, bn);
        // Schur update of the bottom rows (0, 5, 10: lanes 0, 1, 2 at m = 0,
        // 1, 2 respectively)
#pragma unroll
        for (int m = 0; m < 3; ++m)
            if (q == m) {
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) s += Fe[VS_N * VS_N + 3 * VS_N + 3 * m + c] * yprev[c];
                // row 5 m sits at slot m' with q + 4 m' = 5 m
                if (m == 0) bm[0] -= s;
                if (m == 1) bm[1] -= s;
                if (m == 2) bm[2] -= s;
            }
        // all 15 right-hand sides: row q' + 4 m' from lane q'
        double b[VS_N];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const double v0 = quad_bcast<0>(bm[m]), v1 = quad_bcast<1>(bm[m]), v2 = quad_bcast<2>(bm[m]),
                         v3 = quad_bcast<3>(bm[m]);
            if (4 * m + 0 < VS_N) b[4 * m + 0] = v0;
            if (4 * m + 1 < VS_N) b[4 * m + 1] = v1;
            if (4 * m + 2 < VS_N) b[4 * m + 2] = v2;
            if (4 * m + 3 < VS_N) b[4 * m + 3] = v3;
        }
        double y[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int r = has[m] ? q + 4 * m : 0;
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < VS_N; ++c) acc += Fe[r * VS_N + c] * b[c];
            y[m] = acc;
            if (live && has[m]) ys[((int64_t)ez * VS_N + q + 4 * m) * n_lines + line] = acc;
        }
        // y at the top rows 4, 9, 14: lane 0 m = 1, lane 1 m = 2, lane 2 m = 3
        yprev[0] = quad_bcast<0>(y[1]);
        yprev[1] = quad_bcast<1>(y[2]);
        yprev[2] = quad_bcast<2>(y[3]);
    }
    double xb[3] = {0.0, 0.0, 0.0};
    double yn[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) yn[m] = has[m] ? ys[((int64_t)(nz - 1) * VS_N + q + 4 * m) * n_lines + line] : 0.0;
    for (int ez = nz - 1; ez >= 0; --ez) {
        const int e = ex + A.ne0 * (ey + A.ne1 * ez);
        const double* Fe = sFw + ez * HEVI_FAC;
        double x[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) x[m] = yn[m];
        if (ez > 0)
#pragma unroll
            for (int m = 0; m < 4; ++m)
                yn[m] = has[m] ? ys[((int64_t)(ez - 1) * VS_N + q + 4 * m) * n_lines + line] : 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int r = has[m] ? q + 4 * m : 0;
#pragma unroll
            for (int w = 0; w < 3; ++w) x[m] -= Fe[VS_N * VS_N + 3 * r + w] * xb[w];
            if (live && has[m])
                Y[var[m] * A.nnS + (int64_t)e * SRUN + tnode[m]] =
                    (R)(sref<R>(A, var[m], href(A, e, ez, kr[m], tnode[m])) + x[m]);
        }
        // x at the bottom rows 0, 5, 10: lane 0 m = 0, lane 1 m = 1, lane 2 m = 2
        xb[0] = quad_bcast<0>(x[0]);
        xb[1] = quad_bcast<1>(x[1]);
        xb[2] = quad_bcast<2>(x[2]);
    }
}

// the horizontal momenta of the lines with a common matrix: identity
// except the 2 x 2 systems of the interior vertical faces, [1 + s, -s; -s,
// 1 + s] with s = tau lift lam / 2; one thread per (line, variable).  Each
// layer's values are loaded, together with the bottom node of the layer
// above, before anything of the layer is stored, and the next layer's loads
// go out before this layer's stores (the nodes a layer stores are never
// loaded later: the bottom node of a layer above the first belongs to the
// pair below it).
template <typename R>
__global__ __launch_bounds__(256) void k_vmom(const HeviArgs A, const R* B, R* Y, int64_t n_lines)
{
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (id >= 2 * n_lines) return;
    const int v = 1 + (int)(id / n_lines);
    const int64_t line = id % n_lines;
    const int node = (int)(line % (NQ * NQ));
    const int64_t col = line / (NQ * NQ);
    const int i = node % NQ, j = node / NQ;
    const int ex = (int)(col % A.ne0), ey = (int)(col / A.ne0);
    const int nz = A.ne2;
    const double lift = 2.0 / A.h2 * 10.0;
    const R* Bv = B + v * A.nnS;
    R* Yv = Y + v * A.nnS;
    // the line's nodes of layer ez (k = 0..4, k = 0 only in the first
    // layer) and the bottom node of layer ez + 1
    R cur[NQ + 1], nxt[NQ + 1];
    auto load = [&](int ez, R* x) {
        const int64_t eo = (int64_t)(ex + A.ne0 * (ey + A.ne1 * ez)) * SRUN;
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            x[k] = (k > 0 || ez == 0) ? Bv[eo + i + NQ * (j + NQ * k)] : (R)0;
        x[NQ] = ez + 1 < nz ? Bv[eo + (int64_t)A.ne01 * SRUN + i + NQ * j] : (R)0;
    };
    load(0, cur);
    for (int ez = 0; ez < nz; ++ez) {
        if (ez + 1 < nz) load(ez + 1, nxt);
        const int e = ex + A.ne0 * (ey + A.ne1 * ez);
        const int64_t eo = (int64_t)e * SRUN;
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const int tnode = i + NQ * (j + NQ * k);
            if (k == NQ - 1 && ez < nz - 1) {
                const int en = e + A.ne01;
                const int tn = i + NQ * j;
                const int64_t ri = href(A, e, ez, k, tnode), rin = href(A, en, ez + 1, 0, tn);
                const HRef ra = href_tab(A, ri, ez, k), rb = href_tab(A, rin, ez + 1, 0);
                const double lam = ra.c > rb.c ? ra.c : rb.c;
                const double sv = 0.5 * A.tau * lift * lam, al = 1.0 + sv, det = al * al - sv * sv;
                const double xa = (double)cur[k] - sref<R>(A, v, ri);
                const double xbv = (double)cur[NQ] - sref<R>(A, v, rin);
                Yv[eo + tnode] = (R)(sref<R>(A, v, ri) + (al * xa + sv * xbv) / det);
                Yv[(int64_t)en * SRUN + tn] = (R)(sref<R>(A, v, rin) + (sv * xa + al * xbv) / det);
            } else if (!(k == 0 && ez > 0)) {
                Yv[eo + tnode] = cur[k];
            }
        }
#pragma unroll
        for (int q = 0; q <= NQ; ++q) cur[q] = nxt[q];
    }
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
    A.hc = scratch ? scratch + 60 * (int64_t)A.ne2 * hevi_lines(m) : nullptr;
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

size_t hevi_factor_doubles(int nz) { return (size_t)nz * HEVI_FAC; }

hipError_t launch_hevi_solve(cm_model* m, double tau, const void* B, void* Yout, double* scratch, hipStream_t s)
{
    const HeviArgs A = hevi_args(m, tau, scratch);
    const int64_t nl = hevi_lines(m);
    hipLaunchKernelGGL(k_href_table, dim3((unsigned)((A.nref + 255) / 256)), dim3(256), 0, s, A);
    if (m->d_hevi_fac) {
        // every line has the same matrix: factor once per tau (the stream
        // orders it before this and later solves), then apply per line
        if (m->hevi_fac_tau != tau) {
            m->hevi_fac_tau = -1.0;
            hipLaunchKernelGGL(k_vfactor, dim3(1), dim3(64), 0, s, A, m->d_hevi_fac);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            m->hevi_fac_tau = tau;
        }
        const dim3 ga((unsigned)((nl + 63) / 64)), ba(64);
        const dim3 gm((unsigned)((2 * nl + 255) / 256)), bm(256);
        // the whole factor in LDS when it fits a block's share
        int lds_max = 0;
        (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, m->device);
        const size_t whole = sizeof(double) * (size_t)A.ne2 * HEVI_FAC;
        const bool w = whole + 64 <= (size_t)lds_max;
        const double* Fd = m->d_hevi_fac;
        const dim3 g4((unsigned)((4 * nl + 255) / 256)), b4(256);
        if (m->desc.precision == CM_FP64) {
            if (w) hipLaunchKernelGGL(k_vapply4<double>, g4, b4, whole, s, A, Fd, (const double*)B, (double*)Yout, nl);
            else hipLaunchKernelGGL((k_vapply<double, false>), ga, ba, 0, s, A, Fd, (const double*)B, (double*)Yout, nl);
            hipLaunchKernelGGL(k_vmom<double>, gm, bm, 0, s, A, (const double*)B, (double*)Yout, nl);
        } else {
            if (w) hipLaunchKernelGGL(k_vapply4<float>, g4, b4, whole, s, A, Fd, (const float*)B, (float*)Yout, nl);
            else hipLaunchKernelGGL((k_vapply<float, false>), ga, ba, 0, s, A, Fd, (const float*)B, (float*)Yout, nl);
            hipLaunchKernelGGL(k_vmom<float>, gm, bm, 0, s, A, (const float*)B, (float*)Yout, nl);
        }
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((nl + VS_BLOCK / VS_LANES - 1) / (VS_BLOCK / VS_LANES))), block(VS_BLOCK);
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
