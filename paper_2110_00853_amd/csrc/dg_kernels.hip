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
// State layout [var][element][slot], slot = i + 5 j + 25 k, each (variable,
// element) a line-aligned run of SRUN slots (125 nodes, then padding that
// the epilogue fills with zeros so that stores cover whole lines); the
// per-variable bases of a launch come with its parameters and every lane
// addresses its node by a 32-bit byte offset.  Blocks are mapped to elements so
// that each of the eight XCDs walks one contiguous range of elements in a
// tiled order.  Moist viscous models do the saturation adjustment
// once per node and stage: the gradient pass of a step's first stage solves
// it and stores T, the tendency pass reads T and solves for its output
// state (Newton from the input T), which the next stage's passes read.
#include <cmath>

#include "cm_impl.hpp"
#include "fp64_math.hpp"
#include "mlp_common.hpp"
#include "thermo.hpp"

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


// element of a per-variable (or per-word) array whose base comes with the
// launch parameters: with the byte offset in 32 bits the access takes the
// base from scalar registers and one 32-bit vector offset that all the
// variables share, instead of a 64-bit address per lane and variable (the
// offsets fit: the grid size is capped so that 16 x n_nodes < 2^31)
template <typename T> __device__ __forceinline__ __attribute__((address_space(1))) T* gptr(const void* base,
                                                                                         uint32_t byte_off)
{
    return (__attribute__((address_space(1))) T*)((__attribute__((address_space(1))) char*)base + byte_off);
}

// ---------------------------------------------------------------------------
// block -> element: blocks are dealt round-robin to the eight XCDs, and XCD
// x owns the contiguous index range [x q + min(x, r), +q + (x < r)) of the
// n = 8 q + r elements, visited in the order of the grid's traversal table
// (column tiles, so face neighbours share the XCD's L2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int elem_of_block(const KParams& P, int b)
{
    const int n = P.n_elem, q = n >> 3, r = n & 7;
    int x, s;
    if (b < (q << 3)) { x = b & 7; s = b >> 3; }
    else { x = b - (q << 3); s = q; }
    return P.order[x * q + (x < r ? x : r) + s];
}

// neighbour element across face (dir, side), -1 at a wall; ezn receives the
// neighbour's layer index (no integer division per lane)
__device__ __forceinline__ int nbr_elem(const KParams& P, int ex, int ey, int ez, int dir, int side, int& ezn)
{
    int c0 = ex, c1 = ey, c2 = ez;
    if (dir == 0) {
        c0 += side;
        if (c0 < 0 || c0 >= P.ne0) { if (!P.per0) return -1; c0 = c0 < 0 ? P.ne0 - 1 : 0; }
    } else if (dir == 1) {
        c1 += side;
        if (c1 < 0 || c1 >= P.ne1) { if (!P.per1) return -1; c1 = c1 < 0 ? P.ne1 - 1 : 0; }
    } else {
        c2 += side;
        if (c2 < 0 || c2 >= P.ne2) { if (!P.per2) return -1; c2 = c2 < 0 ? P.ne2 - 1 : 0; }
    }
    ezn = c2;
    return c0 + P.ne0 * (c1 + P.ne1 * c2);
}

// (1 + xi_k)/2 of this lane's k, selected from the launch parameters' scalar
// copies: an indexed read of the parameter array would be a vector load,
// and waiting for it waits for every load issued before it (the element's
// own data and its face gathers)
__device__ __forceinline__ double zgll_of(const KParams& P, int k)
{
    double z0 = P.zgll[0], z1 = P.zgll[1], z2 = P.zgll[2], z3 = P.zgll[3], z4 = P.zgll[4];
    // held opaque in scalar registers, or the compiler turns the selects
    // back into one indexed load
    asm volatile("" : "+s"(z0), "+s"(z1), "+s"(z2), "+s"(z3), "+s"(z4));
    double z = z0;
    z = k == 1 ? z1 : z;
    z = k == 2 ? z2 : z;
    z = k == 3 ? z3 : z;
    z = k == 4 ? z4 : z;
    return z;
}

// node height; WARP fixed at compile time in the passes (a flat-mesh
// kernel then carries no per-node height load whose register a later wait
// would have to cover), from the launch parameters elsewhere
template <bool WARP>
__device__ __forceinline__ double node_z(const KParams& P, int e, int ez, int k, int t)
{
    if (WARP) return P.zn[(int64_t)e * NP + t];
    return P.lo2 + ((double)ez + zgll_of(P, k)) * P.h2;
}
__device__ __forceinline__ double node_z(const KParams& P, int e, int ez, int k, int t)
{
    return P.warped ? node_z<true>(P, e, ez, k, t) : node_z<false>(P, e, ez, k, t);
}

__device__ __forceinline__ int ref_index(const KParams& P, int e, int ez, int k, int t)
{
    return P.ref_per_node ? e * NP + t : ez * NQ + k;
}

// the full FP64 value of a stored value x of variable v at reference index
// ri: FP32-bulk storage holds the deviation from the background (so that
// its rounding error scales with the deviation), FP64 storage the value
template <typename R>
__device__ __forceinline__ double full_of(const KParams& P, R x, int v, int ri)
{
    if constexpr (sizeof(R) == 8) return x;
    else return (double)x + (double)P.bg32[(int64_t)v * P.nref + ri];
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
        z = P.lo2 + ((double)ez + zgll_of(P, k)) * P.h2;
    } else {
        const int e = (int)(r / NP), t = (int)(r % NP);
        const int ez = e / (P.ne0 * P.ne1);
        z = node_z(P, e, ez, t / (NQ * NQ), t);
    }
    Th th;
    thermo<MOIST>(Yr[r], Yr[nref + r], Yr[2 * nref + r], Yr[3 * nref + r], Yr[4 * nref + r],
                  MOIST ? Yr[5 * nref + r] : 0.0, z, P.g, P.ice, th);
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
    const R cd = (R)(P.Cs * P.Delta);
    if (P.richardson) {
        const R Ri = N2 * frcp(SS);
        if (Ri > (R)0) {
            // sqrt|S|^2 (1 - Ri/Pr_t)^(1/4) as one fourth root of |S|^4 (1 - Ri/Pr_t)
            const R a = (R)1 - Ri * (R)P.invPrt;
            return a > (R)0 ? cd * cd * fsqrt(fsqrt(SS * SS * a)) : (R)0;
        }
    }
    return cd * cd * fsqrt(SS);
}

// Vreman (eq. vreman-sgs): 2.5 Cs^2 sqrt(B_beta / (u_ij u_ij)) with
// beta_ij = sum_m Dm_m^2 u_i,m u_j,m (Dm the element size over N per
// direction) and B_beta its second principal invariant; the same Richardson
// factor as Smagorinsky-Lilly when enabled.  gu[i][j] = du_i/dx_j.
template <typename R>
__device__ __forceinline__ R vreman(const KParams& P, const R gu[3][3], const R S[3][3], R N2)
{
    const R d2[3] = {(R)(P.h0 * P.h0 * (1.0 / 16.0)), (R)(P.h1 * P.h1 * (1.0 / 16.0)),
                     (R)(P.h2 * P.h2 * (1.0 / 16.0))};
    R aa = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) aa += gu[i][j] * gu[i][j];
    R b[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j)
            b[i][j] = d2[0] * gu[i][0] * gu[j][0] + d2[1] * gu[i][1] * gu[j][1] + d2[2] * gu[i][2] * gu[j][2];
    const R Bb = b[0][0] * b[1][1] + b[0][0] * b[2][2] + b[1][1] * b[2][2] -
                 (b[0][2] * b[0][2] + b[0][1] * b[0][1] + b[1][2] * b[1][2]);
    if (!(aa > (R)0) || !(Bb > (R)0)) return (R)0;
    R nu = (R)(2.5 * P.Cs * P.Cs) * fsqrt(Bb * frcp(aa));
    if (P.richardson) {
        R SS = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) SS += (R)2 * S[a][c] * S[a][c];
        const R Ri = SS > (R)0 ? N2 * frcp(SS) : (R)0;
        if (Ri > (R)0) {
            const R a = (R)1 - Ri * (R)P.invPrt;
            nu = a > (R)0 ? nu * fsqrt(fsqrt(a)) : (R)0;
        }
    }
    return nu;
}

// ---------------------------------------------------------------------------
// face-node tasks: the 6 x 25 face nodes of an element are spread over the
// block's lanes (150 tasks on 128 lanes), so face work runs on dense lanes
// instead of masked passes over the owners.  Task -> (direction, side, own
// node, mirrored node in the neighbour).
// ---------------------------------------------------------------------------
constexpr int NFT = 150;  // face-node tasks per element: 6 faces x 25 nodes

// waves per SIMD the dry flat gradient pass is compiled for (80 VGPRs, no
// spills)
#ifndef CM_MLP_WPE
#define CM_MLP_WPE 1
#endif
#ifndef CM_GRAD_WPE
#define CM_GRAD_WPE 6
#endif

__device__ __forceinline__ void face_task(int task, int& dir, int& sd, int& own, int& nbr)
{
    dir = task / 50;
    const int r = task - 50 * dir;
    sd = r / 25;
    const int f = r - 25 * sd;
    const int a = f % NQ, b = f / NQ;
    const int c = sd ? NQ - 1 : 0, cn = sd ? 0 : NQ - 1;
    if (dir == 0) { own = c + NQ * (a + NQ * b); nbr = cn + NQ * (a + NQ * b); }
    else if (dir == 1) { own = a + NQ * (c + NQ * b); nbr = a + NQ * (cn + NQ * b); }
    else { own = a + NQ * (b + NQ * c); nbr = a + NQ * (b + NQ * cn); }
}

// unit normal (side * J a^dir / |J a^dir|) and lift factor J^s / (J w_N)
template <typename R, bool WARP>
__device__ __forceinline__ void face_normal(const KParams& P, int64_t node, int dir, int side, R n[3], R& lift)
{
    if (WARP) {
        const R* m = (const R*)P.metrics;
        const R a0 = m[(int64_t)(3 * dir + 0) * P.nn + node];
        const R a1 = m[(int64_t)(3 * dir + 1) * P.nn + node];
        const R a2 = m[(int64_t)(3 * dir + 2) * P.nn + node];
        const R invJ = m[9 * P.nn + node];
        const R Js = fsqrt(a0 * a0 + a1 * a1 + a2 * a2);
        const R s = (R)side * frcp(Js);
        n[0] = a0 * s; n[1] = a1 * s; n[2] = a2 * s;
        lift = Js * invJ * (R)(1.0 / WN);
    } else {
        n[0] = dir == 0 ? (R)side : (R)0;
        n[1] = dir == 1 ? (R)side : (R)0;
        n[2] = dir == 2 ? (R)side : (R)0;
        lift = (R)(dir == 0 ? P.lift0 : (dir == 1 ? P.lift1 : P.lift2));
    }
}

// ---------------------------------------------------------------------------
// learned closure: fused BF16-MFMA forward of the 12-64-64-64-2 SiLU network
// for the 64 nodes (rows) of one wave, in the transposed form
// Z^T = W Z_prev^T: the pre-packed weight tiles are the A operands and the
// activations the B operands.  A layer's accumulator tile holds, per lane,
// four consecutive hidden units of one node, which after bias, SiLU and
// conversion to bf16 is the next layer's B operand as it stands, so the
// layers chain in registers with no LDS traffic or barrier between them.
// Inputs sX [128][20] bf16 in LDS (each wave reads only its own rows).
// ---------------------------------------------------------------------------
constexpr int MLP_XS = 20;

typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// SiLU from the hardware exp2 and reciprocal estimates (FP32, a few ulp;
// the result is rounded to bf16 next)
__device__ __forceinline__ float silu_fast(float z)
{
    return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

// SiLU of one accumulator tile (bias included: the accumulation starts from
// it), rounded to bf16 (nearest even)
__device__ __forceinline__ bf16x4 act_bf16(const f32x4& d)
{
    const f32x2 lo = {silu_fast(d[0]), silu_fast(d[1])};
    const f32x2 hi = {silu_fast(d[2]), silu_fast(d[3])};
    const u32x2 u = {__builtin_bit_cast(unsigned, __builtin_convertvector(lo, bf16x2v)),
                     __builtin_bit_cast(unsigned, __builtin_convertvector(hi, bf16x2v))};
    return __builtin_bit_cast(bf16x4, u);
}

// raw outputs (o0, o1) of the node of this lane; row0 = first row of the
// wave.  The wave's four 16-node tiles go through the network CM_MLP_NT at a
// time (fewer live activation and accumulator registers for smaller groups,
// the weight tiles read once per group).
#ifndef CM_MLP_NT
#define CM_MLP_NT 2
#endif
__device__ __forceinline__ void mlp_forward_wave(const KParams& P, const uint16_t (*sX)[MLP_XS], int row0, float& o0,
                                                 float& o1)
{
    constexpr int NTP = CM_MLP_NT;
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, kq = (lane >> 4) * 4;
    const bf16x4* frag = (const bf16x4*)P.mlp_frag;
    const bf16x8s* frag8 = (const bf16x8s*)P.mlp_frag;   // in units of 64 lanes x 8
    const float* bias = P.mlp_bias;
    float v0 = 0.0f, v1 = 0.0f;
#pragma unroll
    for (int g = 0; g < 4; g += NTP) {
        bf16x4 h[4][NTP];  // activations [hidden tile][node tile of the group]
        // layer 1: K = 16 (12 inputs, zero padded)
        bf16x4 xin[NTP];
#pragma unroll
        for (int n = 0; n < NTP; ++n) xin[n] = *(const bf16x4*)&sX[row0 + 16 * (g + n) + r][kq];
#pragma unroll
        for (int ht = 0; ht < 4; ++ht) {
            const bf16x4 a = frag[ht * 64 + lane];
            const f32x4 b = *(const f32x4*)&bias[16 * ht + kq];
#pragma unroll
            for (int n = 0; n < NTP; ++n) h[ht][n] = act_bf16(mfma16(a, xin[n], b));
        }
        // layers 2 and 3: K = 64 as two 32-wide chunks; chunk c of a node
        // tile is the activation tiles 2c and 2c + 1 side by side
#pragma unroll
        for (int layer = 0; layer < 2; ++layer) {
            f32x4 acc[4][NTP];
#pragma unroll
            for (int ht = 0; ht < 4; ++ht) {
                const f32x4 b = *(const f32x4*)&bias[64 * (layer + 1) + 16 * ht + kq];
#pragma unroll
                for (int n = 0; n < NTP; ++n) acc[ht][n] = b;
            }
#pragma unroll
            for (int ht = 0; ht < 4; ++ht)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const bf16x8s a = frag8[((FRAG_L1 + layer * FRAG_L2) / 2 + 2 * ht + c) * 64 + lane];
#pragma unroll
                    for (int n = 0; n < NTP; ++n) acc[ht][n] = mfma32(a, h[2 * c][n], h[2 * c + 1][n], acc[ht][n]);
                }
#pragma unroll
            for (int ht = 0; ht < 4; ++ht)
#pragma unroll
                for (int n = 0; n < NTP; ++n) h[ht][n] = act_bf16(acc[ht][n]);
        }
        // layer 4: one 16-row output tile (rows 0 and 1 real)
        f32x4 out[NTP];
#pragma unroll
        for (int n = 0; n < NTP; ++n) out[n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const bf16x8s a = frag8[((FRAG_L1 + FRAG_L2 + FRAG_L3) / 2 + c) * 64 + lane];
#pragma unroll
            for (int n = 0; n < NTP; ++n) out[n] = mfma32(a, h[2 * c][n], h[2 * c + 1][n], out[n]);
        }
        // lane r < 16 holds rows 0..3 of node 16 nt + r: move outputs 0 and
        // 1 to the lane that owns the node (16 nt + r)
#pragma unroll
        for (int n = 0; n < NTP; ++n) {
            const float s0 = __shfl(out[n][0], r);
            const float s1 = __shfl(out[n][1], r);
            if ((lane >> 4) == g + n) { v0 = s0; v1 = s1; }
        }
    }
    o0 = v0 + bias[192];
    o1 = v1 + bias[193];
}

// softplus log(1 + e^x) = max(x, 0) + log(1 + e^-|x|) in FP32 from the
// hardware exp2 / log2 estimates (log(1 + u) by its series for u < 2^-10)
__device__ __forceinline__ float softplus_f(float x)
{
    const float u = __builtin_amdgcn_exp2f(-1.4426950408889634f * fabsf(x));
    const float l = u < 0x1p-10f ? u * (1.0f - 0.5f * u) : 0.6931471805599453f * __builtin_amdgcn_logf(1.0f + u);
    return fmaxf(x, 0.0f) + l;
}

// neighbour state of one gradient face task
template <typename R, bool MOIST>
struct GradLoad {
    int dir, sd, own, nbl, en, ezn;
    R Yp[MOIST ? 6 : 5];
    double Tq, qcq;  // moist, T_given: the neighbour node's T and condensate
};

template <typename R, bool MOIST>
__device__ __forceinline__ void grad_load(const KParams& P, int task, int e, int ex, int ey,
                                          int ez, GradLoad<R, MOIST>& f)
{
    face_task(task, f.dir, f.sd, f.own, f.nbl);
    f.en = nbr_elem(P, ex, ey, ez, f.dir, f.sd ? 1 : -1, f.ezn);
    const uint32_t soff = (uint32_t)((f.en >= 0 ? f.en : e) * SRUN + f.nbl) * (uint32_t)sizeof(R);
#pragma unroll
    for (int v = 0; v < (MOIST ? 6 : 5); ++v) f.Yp[v] = *gptr<const R>(P.Ys[v], soff);
    if (MOIST && P.T_given) {
        const int64_t nt = (int64_t)(f.en >= 0 ? f.en : e) * run_nodes<double>() + f.nbl;
        f.Tq = P.Tn[nt];
        f.qcq = P.Tn[P.nnT + nt];
    }
}

// lift * (g* - g^-) of one face task into sL[q][task]
template <typename R, bool MOIST, bool WARP, bool ICE>
__device__ __forceinline__ void grad_face(const KParams& P, const GradLoad<R, MOIST>& f, int task, int e,
                                          bool need_thv, bool thv_all_faces, R (*sg)[BLOCK], R (*sL)[NFT])
{
    constexpr int NG = MOIST ? 6 : 5;
    constexpr int GQ = 4, GT = MOIST ? 5 : 4;
    R jump[NG];
    if (f.en >= 0) {
        Th tp;
        double yp[MOIST ? 6 : 5];
        const int rip = ref_index(P, f.en, f.ezn, f.nbl / (NQ * NQ), f.nbl);
#pragma unroll
        for (int v = 0; v < (MOIST ? 6 : 5); ++v) yp[v] = full_of<R>(P, f.Yp[v], v, rip);
        if (MOIST && P.T_given)
            thermo_moist_T(yp[0], yp[1], yp[2], yp[3], yp[4], yp[MOIST ? 5 : 0], f.Tq, f.qcq, ICE, tp);
        else
            thermo<MOIST>(yp[0], yp[1], yp[2], yp[3], yp[4], MOIST ? yp[MOIST ? 5 : 0] : 0.0,
                          node_z<WARP>(P, f.en, f.ezn, f.nbl / (NQ * NQ), f.nbl), P.g, ICE, tp);
        R gp[NG];
        gp[0] = (R)tp.u; gp[1] = (R)tp.v; gp[2] = (R)tp.w; gp[3] = (R)tp.h;
        if (MOIST) gp[GQ] = (R)tp.qt;
        // theta_v: all faces when every component of its gradient is formed,
        // else (flat mesh, only d/dz used) the z faces only
        const bool thv_here = need_thv && (thv_all_faces || f.dir == 2);
        gp[GT] = thv_here ? theta_v<R>(tp) : (R)0;
        R n[3], lift;
        face_normal<R, WARP>(P, (int64_t)e * NP + f.own, f.dir, f.sd ? 1 : -1, n, lift);
#pragma unroll
        for (int q = 0; q < NG; ++q) {
            const R gm = sg[q][f.own];
            jump[q] = lift * ((R)0.5 * (gm + gp[q]) - gm);
        }
        if (!thv_here) jump[GT] = (R)0;
    } else {
#pragma unroll
        for (int q = 0; q < NG; ++q) jump[q] = (R)0;
    }
#pragma unroll
    for (int q = 0; q < NG; ++q) sL[q][task] = jump[q];
}

// ---------------------------------------------------------------------------
// gradient + closure pass
// ---------------------------------------------------------------------------
// FEAT: also export the closure inputs per node (P.feat_out), for training
// ICE: the moist thermodynamics with the ice phase (a compile-time variant,
// so that the liquid-only kernels keep their registers)
template <typename R, bool MOIST, bool WARP, bool MLP, bool FEAT = false, bool ICE = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(MLP ? CM_MLP_WPE : (MOIST || WARP || FEAT ? 1 : CM_GRAD_WPE)))) void k_grad(const KParams P)
{
    constexpr int NV = MOIST ? 6 : 5;
    constexpr int NG = MOIST ? 6 : 5;  // u v w h [qt] thv
    constexpr int GQ = 4, GT = MOIST ? 5 : 4;
    __shared__ R sg[NG][BLOCK];        // gradient variables of the element
    __shared__ R sL[NG][NFT];          // lift * (g* - g^-) per face task

    const int e = elem_of_block(P, blockIdx.x);
    const int t = threadIdx.x;
    const bool act = t < NP;
    const int tt = act ? t : NP - 1;
    const int i = tt % NQ, j = (tt / NQ) % NQ, k = tt / (NQ * NQ);
    const int ex = e % P.ne0, ey = (e / P.ne0) % P.ne1, ez = e / (P.ne0 * P.ne1);
    const int64_t nn = P.nn;
    const int64_t ebase = (int64_t)e * NP;
    const int64_t node = ebase + tt;
    const bool need_thv = ((P.closure == CM_CLOSURE_SMAG || P.closure == CM_CLOSURE_VREMAN) && P.richardson) || MLP;

    GradLoad<R, MOIST> g0;
    grad_load<R, MOIST>(P, t, e, ex, ey, ez, g0);
    // warped meshes: this node's metric terms, loaded at entry so that their
    // latency overlaps phases A and B
    R Ja[3][3], invJ = (R)0;
    if (WARP) {
        const R* m = (const R*)P.metrics;
#pragma unroll
        for (int q = 0; q < 9; ++q) Ja[q / 3][q % 3] = m[(int64_t)q * nn + node];
        invJ = m[9 * nn + node];
    }

    // phase A: thermodynamics and gradient variables into LDS
    Th th;
    {
        double Yv[NV];
        const uint32_t soff = (uint32_t)(e * SRUN + tt) * (uint32_t)sizeof(R);
        const int ri = ref_index(P, e, ez, k, tt);
#pragma unroll
        for (int v = 0; v < NV; ++v) Yv[v] = full_of<R>(P, *gptr<const R>(P.Ys[v], soff), v, ri);
        if (MOIST && P.T_given)
            thermo_moist_T(Yv[0], Yv[1], Yv[2], Yv[3], Yv[4], Yv[MOIST ? 5 : 0],
                           P.Tn[(int64_t)e * run_nodes<double>() + tt],
                           P.Tn[P.nnT + (int64_t)e * run_nodes<double>() + tt], ICE, th);
        else
            thermo<MOIST>(Yv[0], Yv[1], Yv[2], Yv[3], Yv[4], MOIST ? Yv[5] : 0.0, node_z<WARP>(P, e, ez, k, tt), P.g, ICE, th);
    }
    sg[0][t] = (R)th.u; sg[1][t] = (R)th.v; sg[2][t] = (R)th.w; sg[3][t] = (R)th.h;
    if (MOIST) sg[GQ][t] = (R)th.qt;
    // the tendency pass of this stage takes T and the condensate from here instead of
    // repeating the saturation adjustment (every lane stores: whole lines)
    if (MOIST && !P.T_given) {
        const int64_t nt = (int64_t)e * run_nodes<double>() + t;
        __builtin_nontemporal_store(act ? th.T : 0.0, &P.Tn[nt]);
        __builtin_nontemporal_store(act ? th.qc : 0.0, &P.Tn[P.nnT + nt]);
    }
    sg[GT][t] = need_thv ? theta_v<R>(th) : (R)0;
    __syncthreads();

    // phase B: face tasks -> lift * (g* - g^-), centred g* (walls: 0); the
    // first task's neighbour state was loaded at kernel entry
    grad_face<R, MOIST, WARP, ICE>(P, g0, t, e, need_thv, WARP || FEAT, sg, sL);
    if (t + BLOCK < 150) {
        GradLoad<R, MOIST> g1;
        grad_load<R, MOIST>(P, t + BLOCK, e, ex, ey, ez, g1);
        grad_face<R, MOIST, WARP, ICE>(P, g1, t + BLOCK, e, need_thv, WARP || FEAT, sg, sL);
    }
    __syncthreads();

    // phase C: per gradient variable, volume derivative by the 1-D GLL matrix
    // along each direction, chain rule, plus the lifts of the faces this node
    // lies on; the physical gradient G[q][c] = d g_q / d x_c stays in
    // registers.  The variable loop is unrolled (no select chain) with a
    // scheduling barrier after each variable, so that the LDS reads of one
    // variable are not hoisted into the previous one (which would keep every
    // tile in flight and run out of registers)
    const int idx[3] = {i, j, k};
    R nrm[3][3];
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
        const R side = idx[dir] == 0 ? (R)-1 : (R)1;
        if (WARP) {
            const R Js = fsqrt(Ja[dir][0] * Ja[dir][0] + Ja[dir][1] * Ja[dir][1] + Ja[dir][2] * Ja[dir][2]);
            const R s = side * frcp(Js);
            nrm[dir][0] = Ja[dir][0] * s; nrm[dir][1] = Ja[dir][1] * s; nrm[dir][2] = Ja[dir][2] * s;
        } else {
            nrm[dir][0] = dir == 0 ? side : (R)0;
            nrm[dir][1] = dir == 1 ? side : (R)0;
            nrm[dir][2] = dir == 2 ? side : (R)0;
        }
    }
    const bool onf[3] = {i == 0 || i == NQ - 1, j == 0 || j == NQ - 1, k == 0 || k == NQ - 1};
    // face task of this node's face in each direction (task = 50 dir + 25 side + a + 5 b)
    const int ftask[3] = {(i ? 25 : 0) + j + NQ * k, 50 + (j ? 25 : 0) + i + NQ * k, 100 + (k ? 25 : 0) + i + NQ * j};
    R G[NG][3];
#pragma unroll
    for (int q = 0; q < NG; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) G[q][c] = 0;
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        if (q == GT && !WARP && !FEAT) {
            // only d theta_v / dz enters (through N^2): on flat meshes that is
            // the derivative along xi_3 and the lifts of the z faces
            R d2 = 0;
#pragma unroll
            for (int l = 0; l < NQ; ++l) d2 += dmat<R>(k, l) * sg[q][i + NQ * (j + NQ * l)];
            const R jl = sL[q][ftask[2]];
            const R jv = onf[2] ? jl : (R)0;
            R gz = (R)P.r2h2 * d2 + (idx[2] == 0 ? -jv : jv);
            asm volatile("" : "+v"(gz));
            G[q][2] = gz;
            continue;
        }
        R d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
        for (int l = 0; l < NQ; ++l) {
            d0 += dmat<R>(i, l) * sg[q][l + NQ * (j + NQ * k)];
            d1 += dmat<R>(j, l) * sg[q][i + NQ * (l + NQ * k)];
            d2 += dmat<R>(k, l) * sg[q][i + NQ * (j + NQ * l)];
        }
        R gc[3];
        if (WARP) {
#pragma unroll
            for (int c = 0; c < 3; ++c) gc[c] = invJ * (Ja[0][c] * d0 + Ja[1][c] * d1 + Ja[2][c] * d2);
        } else {
            gc[0] = (R)P.r2h0 * d0;
            gc[1] = (R)P.r2h1 * d1;
            gc[2] = (R)P.r2h2 * d2;
        }
        // lifts of the faces this node lies on (read for every node and
        // zeroed off the faces: no divergent branches); on flat meshes the
        // normal is -e_dir / +e_dir on the low / high face
#pragma unroll
        for (int dir = 0; dir < 3; ++dir) {
            const R jl = sL[q][ftask[dir]];
            const R jv = onf[dir] ? jl : (R)0;
            if (WARP) {
#pragma unroll
                for (int c = 0; c < 3; ++c) gc[c] += jv * nrm[dir][c];
            } else {
                gc[dir] += idx[dir] == 0 ? -jv : jv;
            }
        }
        if (FEAT && q == GT && act) {
            // grad theta_v for the closure-input export (only its z part is
            // kept in registers)
            double* f = P.feat_out + node * 16;
            f[12] = (double)gc[0];
            f[13] = (double)gc[1];
            f[14] = (double)gc[2];
        }
        // pin the three results here, so that the arithmetic of this
        // variable is not moved past the next one's LDS reads
        asm volatile("" : "+v"(gc[0]), "+v"(gc[1]), "+v"(gc[2]));
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (q != GT || c == 2) G[q][c] = gc[c];
    }
    R gr[4][3];   // velocity gradient and grad h_tot
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) gr[q][c] = G[q][c];

    // closure and diffusive flux
    R S[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) S[a][b] = (R)0.5 * (gr[a][b] + gr[b][a]);
    R nu = 0, Prt = (R)P.Prt;
    if (P.closure == CM_CLOSURE_CONST) {
        nu = (R)P.nu;
    } else if (P.closure == CM_CLOSURE_VREMAN) {
        const R N2 = P.richardson ? (R)P.g * frcp(sg[GT][t]) * G[GT][2] : (R)0;
        nu = vreman<R>(P, gr, S, N2);
    } else if (P.closure == CM_CLOSURE_SMAG || P.closure == CM_CLOSURE_MLP) {
        const R N2 = P.richardson || MLP ? (R)P.g * frcp(sg[GT][t]) * G[GT][2] : (R)0;
        nu = smagorinsky<R>(P, S, N2);
        if (MLP) {
            // learned closure: standardised inputs (velocity gradient, N^2,
            // filter width, TKE estimate (nu_SL / (0.1 Delta))^2), fused
            // network on the element's nodes, Smagorinsky fallback
            __shared__ uint16_t sX[BLOCK][MLP_XS];
            double raw[12];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) raw[3 * a + b] = (double)gr[a][b];
            raw[9] = (double)N2;
            raw[10] = P.Delta;
            const double kk = (double)nu / (0.1 * P.Delta);
            raw[11] = kk * kk;
            bool out_of_range = false;
#pragma unroll
            for (int q = 0; q < 12; ++q) {
                const double x = (raw[q] - P.mlp_norm[q]) * P.mlp_norm[48 + q];
                if (fabs(x - P.mlp_norm[24 + q]) > P.mlp_norm[36 + q]) out_of_range = true;
                sX[t][q] = f2bf((float)x);
            }
#pragma unroll
            for (int q = 12; q < MLP_XS; ++q) sX[t][q] = 0;
            __syncthreads();
            float o0, o1;
            mlp_forward_wave(P, sX, (threadIdx.x >> 6) * 64, o0, o1);
            double SSd = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) SSd += 2.0 * (double)S[a][b] * (double)S[a][b];
            const double nu_m = P.Delta * P.Delta * sqrt(SSd) * (double)softplus_f(o0);
            const double pr_m = 0.1 + (double)softplus_f(o1);
            const bool fb = P.mlp_fallback_on && (out_of_range || !isfinite(nu_m) || !isfinite(pr_m));
            if (!fb) {
                nu = (R)nu_m;
                Prt = (R)pr_m;
            }
            const unsigned long long nfb = __popcll(__ballot(fb && act));
            if ((threadIdx.x & 63) == 0 && nfb) atomicAdd(P.mlp_fallbacks, nfb);
        }
    }
    if (FEAT && !MLP && act) {
        // closure inputs for training: grad u (9), N^2, Delta, TKE estimate
        // (nu_SL / (0.1 Delta))^2, grad theta_v (3), theta_v
        double* f = P.feat_out + node * 16;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) f[3 * a + b] = (double)gr[a][b];
        f[9] = P.g / (double)sg[GT][t] * (double)G[GT][2];
        f[10] = P.Delta;
        const double kk = (double)nu / (0.1 * P.Delta);
        f[11] = kk * kk;
        f[15] = (double)sg[GT][t];
    }
    const R rho = (R)th.rho;
    const R Dt = MLP ? nu * frcp(Prt) : nu * (R)P.invPrt;
    const R c2 = (R)(-2.0) * rho * nu;
    R w[14] = {};
    w[0] = c2 * S[0][0]; w[1] = c2 * S[1][1]; w[2] = c2 * S[2][2];
    w[3] = c2 * S[0][1]; w[4] = c2 * S[0][2]; w[5] = c2 * S[1][2];
    const R u0 = sg[0][t], u1 = sg[1][t], u2 = sg[2][t];  // (R) u, v, w of this node
    const R rDt = rho * Dt;
    w[6] = u0 * w[0] + u1 * w[3] + u2 * w[4] - rDt * gr[3][0];
    w[7] = u0 * w[3] + u1 * w[1] + u2 * w[5] - rDt * gr[3][1];
    w[8] = u0 * w[4] + u1 * w[5] + u2 * w[2] - rDt * gr[3][2];
    if (MOIST) {
        w[9] = -rDt * G[GQ][0];
        w[10] = -rDt * G[GQ][1];
        w[11] = -rDt * G[GQ][2];
    }
    // subsidence needs d/dz of h_tot (and q_t) in the tendency pass
    constexpr int SB = MOIST ? 12 : 9;
    w[SB] = gr[3][2];
    if (MOIST) w[SB + 1] = G[GQ][2];
    const int nw = SB + (P.subsidence ? (MOIST ? 2 : 1) : 0);
    // every lane stores (the three beyond the element write the padding), so
    // that each wave writes whole cache lines
#pragma unroll
    for (int q = 0; q < 14; ++q)
        if (q < nw)
            __builtin_nontemporal_store(act ? w[q] : (R)0,
                                        gptr<R>(P.F2s[q], (uint32_t)(e * run_nodes<R>() + t) * (uint32_t)sizeof(R)));
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

// normal inviscid flux n.F1 from primitive quantities
template <typename R, bool MOIST>
__device__ __forceinline__ void flux1_normal(R rho, const R u[3], R pp, R ep, R rq, const R n[3], R out[])
{
    const R un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
    const R m = rho * un;
    out[0] = m;
    out[1] = m * u[0] + pp * n[0];
    out[2] = m * u[1] + pp * n[1];
    out[3] = m * u[2] + pp * n[2];
    out[4] = ep * un;
    if (MOIST) out[5] = rq * un;
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

// normal component of a neighbour's stored diffusive flux on a flat mesh,
// n = side e_dir, from the dir column of the flux (the words face_load keeps)
template <typename R, bool MOIST>
__device__ __forceinline__ void f2_normal_axis(const R* wq, const R u[3], R side, R out[])
{
    out[0] = MOIST ? side * wq[4] : (R)0;
    out[1] = side * wq[0];
    out[2] = side * wq[1];
    out[3] = side * wq[2];
    out[4] = side * wq[3];
    if (MOIST) {
        out[1] += out[0] * u[0];
        out[2] += out[0] * u[1];
        out[3] += out[0] * u[2];
        out[5] = out[0];
    }
}

// whether the tendency pass keeps the own nodes' velocity and sound speed in
// LDS for the face tasks (moist inviscid: no carried temperature to
// recompute them from; FP32 storage: LDS is not the limit) or recomputes them
template <typename R, bool MOIST, bool VISC> constexpr bool tend_keeps_p()
{
    return (MOIST && !VISC) || sizeof(R) == 4;
}

// data of one face task: the neighbour's state, diffusive flux (all words on
// warped meshes; on flat meshes only the column of the face direction:
// tau_{x,dir}, tau_{y,dir}, tau_{z,dir}, energy and water flux along dir)
// and reference pressure, loaded before they are needed; the own node's
// state comes from LDS
template <typename R, bool MOIST, bool WARP, bool VISC>
struct FaceLoad {
    static constexpr int NV = MOIST ? 6 : 5;
    static constexpr int NW = MOIST ? 12 : 9;
    static constexpr int NWF = WARP ? NW : (MOIST ? 5 : 4);
    int dir, sd, own, nbl, en, ezn;
    R Yp[NV], wp[VISC ? NWF : 1];
    float bgp[sizeof(R) == 4 ? NV : 1];  // FP32 storage: the neighbour node's background
    double prp;
    double Tq, qcq;  // moist viscous: T and condensate of the neighbour node (of this node on a wall)
    double To, qco;  // moist viscous: T and condensate of the own node
};

template <typename R, bool MOIST, bool WARP, bool VISC>
__device__ __forceinline__ void face_load(const KParams& P, const R* __restrict__ F2,
                                          int task, int e, int ex, int ey, int ez,
                                          FaceLoad<R, MOIST, WARP, VISC>& f)
{
    constexpr int NV = FaceLoad<R, MOIST, WARP, VISC>::NV;
    constexpr int NW = FaceLoad<R, MOIST, WARP, VISC>::NW;
    face_task(task, f.dir, f.sd, f.own, f.nbl);
    f.en = nbr_elem(P, ex, ey, ez, f.dir, f.sd ? 1 : -1, f.ezn);
    const int eo = f.en >= 0 ? f.en : e;  // walls read their own node twice
    const int ezo = f.en >= 0 ? f.ezn : ez;
    const uint32_t soff = (uint32_t)(eo * SRUN + f.nbl) * (uint32_t)sizeof(R);  // state slot, bytes
    const int64_t npf = (int64_t)eo * run_nodes<R>() + f.nbl;  // in the padded F2 runs
#pragma unroll
    for (int v = 0; v < NV; ++v) f.Yp[v] = *gptr<const R>(P.Ys[v], soff);
    if (VISC) {
        if (WARP) {
#pragma unroll
            for (int q = 0; q < NW; ++q) f.wp[q] = F2[q * P.nnf + npf];
        } else {
            // symmetric tau stored as xx yy zz xy xz yz: tau_{c,dir} is word
            // c when c = dir, else 2 + c + dir
            const int d = f.dir;
#pragma unroll
            for (int c = 0; c < 3; ++c) f.wp[c] = F2[(c == d ? c : 2 + c + d) * P.nnf + npf];
            f.wp[3] = F2[(6 + d) * P.nnf + npf];
            if (MOIST) f.wp[4] = F2[(9 + d) * P.nnf + npf];
        }
    }
    // reference pressure of the neighbour node; on a wall the neighbour slot
    // holds this element's mirrored node, and the flux needs this node's
    const int rn = f.en >= 0 ? f.nbl : f.own;
    const int rin = ref_index(P, eo, ezo, rn / (NQ * NQ), rn);
    f.prp = P.pr[rin];
    if constexpr (sizeof(R) == 4) {
#pragma unroll
        for (int v = 0; v < NV; ++v) f.bgp[v] = P.bg32[(int64_t)v * P.nref + rin];
    }
    if (MOIST && VISC) {
        const int64_t nt = (int64_t)eo * run_nodes<double>() + rn;
        f.Tq = P.Tn[nt];
        f.qcq = P.Tn[P.nnT + nt];
        const int64_t no = (int64_t)e * run_nodes<double>() + f.own;
        f.To = P.Tn[no];
        f.qco = P.Tn[P.nnT + no];
    }
}

// Dissipative part of the Roe and HLLC numerical fluxes for dry air (Sect.
// 3.1), written as D with n.F1* = (n.F1^- + n.F1^+)/2 - D/2 (Rusanov: D =
// lambda (Y^+ - Y^-)).  FP64 from the two sides' thermodynamics; the
// reference pressure cancels from D (it is continuous at the node).
//
// Roe: D = sum_k |lambda_k| alpha_k r_k over the two acoustic waves, the
// entropy wave and the shear wave of the sqrt(rho)-weighted average state.
// The internal energy counts from T_0, so rho e_tot + rho c_vd T_0 is the
// ideal-gas total energy of the textbook Roe matrix: its sound speed is
// c^2 = (R_d/c_vd)(H + c_vd T_0 - |u|^2/2 - g z), and the energy components
// of the eigenvectors are the textbook ones less c_vd T_0.
__device__ __forceinline__ void roe_dissipation(const Th& a, const Th& b, double phi, const double n[3], double D[5])
{
    const double sa = fsqrt(a.rho), sb = fsqrt(b.rho);
    const double inv = frcp(sa + sb);
    const double wa = sa * inv, wb = sb * inv, rh = sa * sb;
    const double uh[3] = {wa * a.u + wb * b.u, wa * a.v + wb * b.v, wa * a.w + wb * b.w};
    const double du[3] = {b.u - a.u, b.v - a.v, b.w - a.w};
    const double Hh = wa * a.h + wb * b.h;
    const double q2 = uh[0] * uh[0] + uh[1] * uh[1] + uh[2] * uh[2];
    const double c2 = (Phys::Rd / Phys::cvd) * (Hh + Phys::cvd * Phys::T0 - 0.5 * q2 - phi);
    const double ch = fsqrt(c2), ic2 = frcp(c2);
    const double unh = uh[0] * n[0] + uh[1] * n[1] + uh[2] * n[2];
    const double dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
    const double dp = b.p - a.p;
    const double a1 = 0.5 * (dp - rh * ch * dun) * ic2;
    const double a2 = (b.rho - a.rho) - dp * ic2;
    const double a3 = 0.5 * (dp + rh * ch * dun) * ic2;
    const double l1 = fabs(unh - ch), l2 = fabs(unh), l3 = fabs(unh + ch);
    const double w1 = l1 * a1, w2 = l2 * a2, w3 = l3 * a3, ws = l2 * rh;
    D[0] = w1 + w2 + w3;
#pragma unroll
    for (int c = 0; c < 3; ++c) D[1 + c] = (w1 + w2 + w3) * uh[c] + (w3 - w1) * ch * n[c] + ws * (du[c] - dun * n[c]);
    D[4] = (w1 + w3) * Hh + (w3 - w1) * ch * unh + w2 * (0.5 * q2 + phi - Phys::cvd * Phys::T0) +
           ws * (uh[0] * du[0] + uh[1] * du[1] + uh[2] * du[2] - unh * dun);
}

// HLLC with Davis wave-speed bounds S_a = min(u_n - c), S_b = max(u_n + c)
// over the two sides and the contact speed S* from the jump conditions; the
// flux of the side whose fan holds the node direction, f_K + S_K (U*_K -
// U_K), with U*_K = rho_K (S_K - u_nK)/(S_K - S*) (1, u_K + (S* - u_nK) n,
// e_K + (S* - u_nK)(S* + p_K/(rho_K (S_K - u_nK)))).  Returned as D = f^- +
// f^+ - 2 F* (normal inviscid fluxes with the full pressure).
__device__ __forceinline__ void hllc_dissipation(const Th& a, const Th& b, const double n[3], double D[5])
{
    const double una = a.u * n[0] + a.v * n[1] + a.w * n[2];
    const double unb = b.u * n[0] + b.v * n[1] + b.w * n[2];
    double fa[5], fb[5];
    fa[0] = a.rho * una; fb[0] = b.rho * unb;
    fa[1] = fa[0] * a.u + a.p * n[0]; fb[1] = fb[0] * b.u + b.p * n[0];
    fa[2] = fa[0] * a.v + a.p * n[1]; fb[2] = fb[0] * b.v + b.p * n[1];
    fa[3] = fa[0] * a.w + a.p * n[2]; fb[3] = fb[0] * b.w + b.p * n[2];
    fa[4] = (a.rho * a.e + a.p) * una; fb[4] = (b.rho * b.e + b.p) * unb;
    const double Sa = fmin(una - a.c, unb - b.c), Sb = fmax(una + a.c, unb + b.c);
    double F[5];
    if (Sa >= 0.0) {
#pragma unroll
        for (int v = 0; v < 5; ++v) F[v] = fa[v];
    } else if (Sb <= 0.0) {
#pragma unroll
        for (int v = 0; v < 5; ++v) F[v] = fb[v];
    } else {
        const double ma = a.rho * (Sa - una), mb = b.rho * (Sb - unb);
        const double Ss = (b.p - a.p + una * ma - unb * mb) * frcp(ma - mb);
        const bool left = Ss >= 0.0;
        const Th& k = left ? a : b;
        const double S = left ? Sa : Sb, un = left ? una : unb, mk = left ? ma : mb;
        const double fac = mk * frcp(S - Ss);
        const double sh = Ss - un;
        const double Uk[5] = {k.rho, k.rho * k.u, k.rho * k.v, k.rho * k.w, k.rho * k.e};
        const double Us[5] = {fac, fac * (k.u + sh * n[0]), fac * (k.v + sh * n[1]), fac * (k.w + sh * n[2]),
                              fac * (k.e + sh * (Ss + k.p * frcp(mk)))};
#pragma unroll
        for (int v = 0; v < 5; ++v) F[v] = (left ? fa[v] : fb[v]) + S * (Us[v] - Uk[v]);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) D[v] = fa[v] + fb[v] - 2.0 * F[v];
}

// numerical flux of one face task; writes lift (n.F^- - n.F^*) over the
// task's own-node entries of sG (the divergence is already done)
template <typename R, bool MOIST, bool WARP, bool VISC, int VAR>
__device__ __forceinline__ void face_flux(const KParams& P, const FaceLoad<R, MOIST, WARP, VISC>& f, int e, int ez,
                                          R (*sG)[NP], R (*sP)[BLOCK], R (*sY)[BLOCK])
{
    // VAR: the numerical flux of a dry model (0 Rusanov, 1 Roe, 2 HLLC); for
    // a moist model 1 selects the ice phase
    constexpr int FLUX = MOIST ? 0 : VAR;
    constexpr bool ICE = MOIST && VAR == 1;
    constexpr int NV = MOIST ? 6 : 5;
    const int64_t nn = P.nn;
    const int dir = f.dir, sd = f.sd, own = f.own, nbl = f.nbl, en = f.en;
    const int side = sd ? 1 : -1;
    const int64_t onode = (int64_t)e * NP + own;
    R n[3], lift;
    face_normal<R, WARP>(P, onode, dir, side, n, lift);
    const R cJ = WARP ? ((const R*)P.metrics)[9 * nn + onode] * (R)(1.0 / WN) : (R)(1.0 / WN);
    R Ym[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Ym[v] = sY[v][own];
    // full own and neighbour states in FP64 (FP32-bulk stores deviations
    // from the background; on a wall the neighbour slot is this node)
    const int rio = ref_index(P, e, ez, own / (NQ * NQ), own);
    double ym[NV], yp[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        ym[v] = full_of<R>(P, Ym[v], v, rio);
        // the neighbour's background was loaded with its state (on a wall
        // the neighbour slot is this node, and so is the background read)
        if constexpr (sizeof(R) == 8) yp[v] = f.Yp[v];
        else yp[v] = (double)f.Yp[v] + (double)f.bgp[v];
    }
    // own node's velocity and sound speed: from LDS in the moist inviscid
    // case (the saturation adjustment is too costly to repeat) and with FP32
    // storage (LDS is not the limit there); recomputed from the own state in
    // the FP64 dry and moist viscous cases (the same FP64 arithmetic as phase
    // A, with the moist temperature that phase A used, so the same values,
    // and 4 KB less LDS per block)
    // (Roe and HLLC need the own node's pressure and enthalpy: always recomputed)
    constexpr bool KEEP_P = tend_keeps_p<R, MOIST, VISC>() && FLUX == 0;
    Th to;
    R um[3], cm;
    if (KEEP_P) {
        um[0] = sP[0][own]; um[1] = sP[1][own]; um[2] = sP[2][own];
        cm = sP[3][own];
    } else {
        if (MOIST)
            thermo_moist_T(ym[0], ym[1], ym[2], ym[3], ym[4], ym[NV - 1], f.To, f.qco, ICE, to);
        else
            thermo<false>(ym[0], ym[1], ym[2], ym[3], ym[4], 0.0, node_z<WARP>(P, e, ez, own / (NQ * NQ), own), P.g,
                          ICE, to);
        um[0] = (R)to.u; um[1] = (R)to.v; um[2] = (R)to.w;
        cm = (R)to.c;
    }
    const R unm = um[0] * n[0] + um[1] * n[1] + um[2] * n[2];
    R liftFm[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) liftFm[v] = (R)side * sG[v * 3 + dir][own] * cJ;
    R contrib[NV];
    if (en >= 0) {
        const int ezn = f.ezn;
        const int kn = nbl / (NQ * NQ);
        Th tp;
        if (MOIST && VISC)
            thermo_moist_T(yp[0], yp[1], yp[2], yp[3], yp[4], yp[NV - 1], f.Tq, f.qcq, ICE, tp);
        else
            thermo<MOIST>(yp[0], yp[1], yp[2], yp[3], yp[4], MOIST ? yp[NV - 1] : 0.0,
                          node_z<WARP>(P, en, ezn, kn, nbl), P.g, ICE, tp);
        const R up[3] = {(R)tp.u, (R)tp.v, (R)tp.w};
        R fp[NV];
        flux1_normal<R, MOIST>((R)tp.rho, up, (R)(tp.p - f.prp), (R)(tp.rho * tp.e + tp.p), (R)(tp.rho * tp.qt), n,
                               fp);
        if (VISC) {
            R fp2[NV];
            if (WARP) f2_normal<R, MOIST>(f.wp, up, n, fp2);
            else f2_normal_axis<R, MOIST>(f.wp, up, (R)side, fp2);
#pragma unroll
            for (int v = 0; v < NV; ++v) fp[v] += fp2[v];
        }
        if (FLUX == 0) {
            const R unp = up[0] * n[0] + up[1] * n[1] + up[2] * n[2];
            const R lm = fabs(unm) + cm, lp = fabs(unp) + (R)tp.c;
            const R lam = lm > lp ? lm : lp;
#pragma unroll
            for (int v = 0; v < NV; ++v)
                contrib[v] = (R)0.5 * (liftFm[v] - lift * fp[v]) -
                             (R)0.5 * lift * lam * (sizeof(R) == 8 ? Ym[v] - f.Yp[v] : (R)(ym[v] - yp[v]));
        } else {
            const double nd[3] = {(double)n[0], (double)n[1], (double)n[2]};
            double D[5];
            if (FLUX == 1) roe_dissipation(to, tp, P.g * node_z<WARP>(P, e, ez, own / (NQ * NQ), own), nd, D);
            else hllc_dissipation(to, tp, nd, D);
#pragma unroll
            for (int v = 0; v < NV; ++v) contrib[v] = (R)0.5 * (liftFm[v] - lift * fp[v]) + (R)0.5 * lift * (R)D[v];
        }
    } else {
        // reflecting ghost u+ = u- - 2 (n.u-) n with rho, rho e, rho q
        // mirrored: the Rusanov flux of (Y-, ghost) plus the prescribed wall
        // diffusive flux
        // (without KEEP_P, to already holds this node's thermodynamics; on a
        // wall the neighbour slot's T and condensate are this node's)
        Th tm = to;
        if (KEEP_P && !MOIST)
            thermo<false>(ym[0], ym[1], ym[2], ym[3], ym[4], 0.0, node_z<WARP>(P, e, ez, own / (NQ * NQ), own), P.g,
                          ICE, tm);
        else if (KEEP_P && MOIST && VISC)
            thermo_moist_T(ym[0], ym[1], ym[2], ym[3], ym[4], ym[NV - 1], f.Tq, f.qcq, ICE, tm);
        else if (MOIST && !VISC)
            thermo<MOIST>(ym[0], ym[1], ym[2], ym[3], ym[4], ym[NV - 1], node_z<WARP>(P, e, ez, own / (NQ * NQ), own),
                          P.g, ICE, tm);
        const R rho = sizeof(R) == 8 ? Ym[0] : (R)ym[0];
        const R pp = (R)(tm.p - f.prp), ep = (R)(tm.rho * tm.e + tm.p);
        const R rq = MOIST ? (sizeof(R) == 8 ? Ym[NV - 1] : (R)ym[NV - 1]) : (R)0;
        const R ug[3] = {um[0] - (R)2 * unm * n[0], um[1] - (R)2 * unm * n[1], um[2] - (R)2 * unm * n[2]};
        R f1m[NV], f1g[NV];
        flux1_normal<R, MOIST>(rho, um, pp, ep, rq, n, f1m);
        flux1_normal<R, MOIST>(rho, ug, pp, ep, rq, n, f1g);
        const R lam = fabs(unm) + cm;
        R jumpY[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) jumpY[v] = (R)0;
        const R mn = sizeof(R) == 8 ? Ym[1] * n[0] + Ym[2] * n[1] + Ym[3] * n[2]
                                    : (R)ym[1] * n[0] + (R)ym[2] * n[1] + (R)ym[3] * n[2];
        jumpY[1] = (R)2 * mn * n[0];
        jumpY[2] = (R)2 * mn * n[1];
        jumpY[3] = (R)2 * mn * n[2];
        R f2s[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) f2s[v] = (R)0;
        if (VISC && P.sfc_flux && dir == 2 && sd == 0) {
            // prescribed upward surface fluxes; the outward normal is -z
            const double qf = MOIST ? P.qt_flux : 0.0;
            f2s[4] = (R)(-(double)rho * (Phys::cpd * P.theta_flux + Phys::Lv0 * qf));
            if (MOIST) {
                f2s[0] = (R)(-(double)rho * qf);
                f2s[NV - 1] = f2s[0];
            }
        }
        if (FLUX == 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
                contrib[v] = liftFm[v] - lift * ((R)0.5 * (f1m[v] + f1g[v]) + (R)0.5 * lam * jumpY[v] + f2s[v]);
        } else {
            // the ghost: same density, pressure, enthalpy and sound speed,
            // mirrored velocity
            Th tg = tm;
            const double und = tm.u * (double)n[0] + tm.v * (double)n[1] + tm.w * (double)n[2];
            tg.u = tm.u - 2.0 * und * (double)n[0];
            tg.v = tm.v - 2.0 * und * (double)n[1];
            tg.w = tm.w - 2.0 * und * (double)n[2];
            const double nd[3] = {(double)n[0], (double)n[1], (double)n[2]};
            double D[5];
            if (FLUX == 1) roe_dissipation(tm, tg, P.g * node_z<WARP>(P, e, ez, own / (NQ * NQ), own), nd, D);
            else hllc_dissipation(tm, tg, nd, D);
#pragma unroll
            for (int v = 0; v < NV; ++v)
                contrib[v] = liftFm[v] - lift * ((R)0.5 * (f1m[v] + f1g[v]) - (R)0.5 * (R)D[v] + f2s[v]);
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) sG[v * 3 + dir][own] = contrib[v];
}

// own-node data of one element
template <typename R, bool MOIST, bool WARP, bool VISC, int MODE>
struct OwnLoad {
    static constexpr int NV = MOIST ? 6 : 5;
    static constexpr int NW = MOIST ? 12 : 9;
    static constexpr int NWS = NW + (MOIST ? 2 : 1);  // with the subsidence words
    R Yr[NV];
    float bg[sizeof(R) == 4 ? NV : 1];  // FP32 storage: the node's background
    R w[VISC ? NWS : 1];
    R Jam[WARP ? 10 : 1];  // J a^d (9) and 1/J
    double pr, rr;
    double T, qc;  // moist viscous: T and condensate from earlier in the stage
};

template <typename R, bool MOIST, bool WARP, bool VISC, int MODE>
__device__ __forceinline__ void own_load(const KParams& P, int e, int ez, int tt,
                                         OwnLoad<R, MOIST, WARP, VISC, MODE>& o)
{
    using O = OwnLoad<R, MOIST, WARP, VISC, MODE>;
    const int64_t nn = P.nn;
    const int64_t node = (int64_t)e * NP + tt;
    const uint32_t soff = (uint32_t)(e * SRUN + tt) * (uint32_t)sizeof(R);  // byte offset in the state buffers
#pragma unroll
    for (int v = 0; v < O::NV; ++v) o.Yr[v] = *gptr<const R>(P.Ys[v], soff);
    if (VISC) {
        const int nw = P.subsidence ? O::NWS : O::NW;
        const uint32_t foff = (uint32_t)(e * run_nodes<R>() + tt) * (uint32_t)sizeof(R);
#pragma unroll
        for (int q = 0; q < O::NWS; ++q) o.w[q] = q < nw ? *gptr<const R>(P.F2s[q], foff) : (R)0;
    }

    const int ri = ref_index(P, e, ez, tt / (NQ * NQ), tt);
    o.pr = P.pr[ri];
    o.rr = P.rhor[ri];
    if constexpr (sizeof(R) == 4) {
#pragma unroll
        for (int v = 0; v < O::NV; ++v) o.bg[v] = P.bg32[(int64_t)v * P.nref + ri];
    }
    if (MOIST && VISC) {
        o.T = P.Tn[(int64_t)e * run_nodes<double>() + tt];
        o.qc = P.Tn[P.nnT + (int64_t)e * run_nodes<double>() + tt];
    }
    if (WARP) {
        const R* m = (const R*)P.metrics;
#pragma unroll
        for (int q = 0; q < 10; ++q) o.Jam[q] = m[(int64_t)q * nn + node];
    }
}

// the tendency of one element from its loaded data: thermodynamics ->
// contravariant flux in LDS -> divergence -> face tasks -> sources ->
// epilogue.  MODE 0: out = R; MODE 1: LSRK stage; MODE 2: first LSRK stage
// (A = 0, dQ not read).  The second face task (t + BLOCK < 150) is loaded
// just before it is needed: loaded earlier, its registers stay live through
// the divergence and cost a wave per SIMD (measured slower).
template <typename R, bool MOIST, bool WARP, bool VISC, int MODE, int VAR>
__device__ __forceinline__ void tend_element(const KParams& P, int e, int t,
                                             const OwnLoad<R, MOIST, WARP, VISC, MODE>& o,
                                             const FaceLoad<R, MOIST, WARP, VISC>& ft0, R dval,
                                             R (*sG)[NP], R (*sP)[BLOCK], R (*sY)[BLOCK], R* sD,
                                             const R* __restrict__ F2, R A, R B, R dt)
{
    constexpr bool ICE = MOIST && VAR == 1;
    constexpr int NV = MOIST ? 6 : 5;
    constexpr int NW = MOIST ? 12 : 9;
    const bool act = t < NP;
    const int tt = act ? t : NP - 1;
    const int i = tt % NQ, j = (tt / NQ) % NQ, k = tt / (NQ * NQ);
    const int ex = e % P.ne0, ey = (e / P.ne0) % P.ne1, ez = e / (P.ne0 * P.ne1);
    const double z = node_z<WARP>(P, e, ez, k, tt);
    double rho_d, mom_d[3];
    {
        Th th;
        double y[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if constexpr (sizeof(R) == 8) y[v] = o.Yr[v];
            else y[v] = (double)o.Yr[v] + (double)o.bg[v];
        }
        if (MOIST && VISC)
            thermo_moist_T(y[0], y[1], y[2], y[3], y[4], y[NV - 1], o.T, o.qc, ICE, th);
        else
            thermo<MOIST>(y[0], y[1], y[2], y[3], y[4], MOIST ? y[NV - 1] : 0.0, z, P.g, ICE, th);
        rho_d = th.rho;
        mom_d[0] = y[1]; mom_d[1] = y[2]; mom_d[2] = y[3];
        R F[NV][3];
        flux1<R, MOIST>(th, o.pr, F);
        const R um[3] = {(R)th.u, (R)th.v, (R)th.w};
        if (tend_keeps_p<R, MOIST, VISC>()) {
            sP[0][t] = um[0]; sP[1][t] = um[1]; sP[2][t] = um[2];
            sP[3][t] = (R)th.c;
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) sY[v][t] = o.Yr[v];
        if (VISC) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const R nd[3] = {d == 0 ? (R)1 : (R)0, d == 1 ? (R)1 : (R)0, d == 2 ? (R)1 : (R)0};
                R f2[NV];
                f2_normal<R, MOIST>(o.w, um, nd, f2);
#pragma unroll
                for (int v = 0; v < NV; ++v) F[v][d] += f2[v];
            }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                R G;
                if (WARP) G = o.Jam[3 * d] * F[v][0] + o.Jam[3 * d + 1] * F[v][1] + o.Jam[3 * d + 2] * F[v][2];
                else G = (R)(d == 0 ? P.r2h0 : (d == 1 ? P.r2h1 : P.r2h2)) * F[v][d];
                if (act) sG[v * 3 + d][t] = G;
            }
    }
    // the differentiation matrix into LDS column by column, D[r][c] at
    // sD[5c + r]: the five rows a wave reads for one c are consecutive words,
    // in distinct banks (its load was issued first, so phase B waits for no
    // global load)
    if (t < NQ * NQ) sD[(t % NQ) * NQ + t / NQ] = dval;
    __syncthreads();

    // phase B: strong-form divergence with the 1-D GLL matrix, one variable
    // at a time: each variable's sum is pinned before the next variable's
    // LDS reads, so that the compiler does not keep every tile in flight
    R Rv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        R s = 0;
#pragma unroll
        for (int l = 0; l < NQ; ++l) {
            s += sD[l * NQ + i] * sG[v * 3 + 0][l + NQ * (j + NQ * k)];
            s += sD[l * NQ + j] * sG[v * 3 + 1][i + NQ * (l + NQ * k)];
            s += sD[l * NQ + k] * sG[v * 3 + 2][i + NQ * (j + NQ * l)];
        }
        asm volatile("" : "+v"(s));
        Rv[v] = -s;
    }
    __syncthreads();


    // phase C: face tasks.  lift (n.F^- - n.F^*): n.F^- comes from the
    // contravariant flux already in LDS (lift n.F = side G^dir / (J w_N)).
    // The first task's loads were issued at kernel entry (ft0).
    face_flux<R, MOIST, WARP, VISC, VAR>(P, ft0, e, ez, sG, sP, sY);
    if (t + BLOCK < NFT) {
        FaceLoad<R, MOIST, WARP, VISC> ft1;
        face_load<R, MOIST, WARP, VISC>(P, F2, t + BLOCK, e, ex, ey, ez, ft1);
        face_flux<R, MOIST, WARP, VISC, VAR>(P, ft1, e, ez, sG, sP, sY);
    }
    __syncthreads();

    // phase D: gather the face terms of this node, metric factor, sources
    // the stage's dQ is loaded only now: loaded with the rest of the own
    // data at entry, its registers stay live through phases A to C
    // (120 instead of 110 VGPRs, 1 % slower)
    R dqv[MODE == 1 ? NV : 1];
    if (MODE == 1) {
        const uint32_t doff = (uint32_t)(e * SRUN + tt) * (uint32_t)sizeof(R);
#pragma unroll
        for (int v = 0; v < NV; ++v) dqv[v] = __builtin_nontemporal_load(gptr<const R>(P.dQs[v], doff));
    }
    const int idx[3] = {i, j, k};
    if (WARP) {
        const R invJ = o.Jam[9];
#pragma unroll
        for (int v = 0; v < NV; ++v) Rv[v] *= invJ;
    }
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
        // read for every node, added on the face nodes only (no divergent branch)
        const bool on = idx[dir] == 0 || idx[dir] == NQ - 1;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const R fv = sG[v * 3 + dir][tt];
            Rv[v] += on ? fv : (R)0;
        }
    }
    Rv[3] -= (R)((rho_d - o.rr) * P.g);
    if (P.f_cor != 0.0) {
        Rv[1] += (R)(P.f_cor * (mom_d[1] - rho_d * P.v_g));
        Rv[2] -= (R)(P.f_cor * (mom_d[0] - rho_d * P.u_g));
    }
    if (P.sponge && z > P.sp_zs) {
        const double zeta = (z - P.sp_zs) * P.sp_inv;
        const double tau = P.sp_alpha * pow(sin(0.5 * M_PI * zeta), P.sp_gamma);
        Rv[1] -= (R)(tau * (mom_d[0] - rho_d * P.sp_u0));
        Rv[2] -= (R)(tau * (mom_d[1] - rho_d * P.sp_u1));
        Rv[3] -= (R)(tau * (mom_d[2] - rho_d * P.sp_u2));
    }
    if (VISC && P.subsidence) {
        const double zz = z < P.sub_ztop ? z : P.sub_ztop;
        const double ws = -P.sub_w0 * sin(M_PI * zz * P.sub_inv);
        const R rws = (R)(rho_d * ws);
        Rv[4] -= rws * o.w[NW];
        if (MOIST) Rv[NV - 1] -= rws * o.w[NW + 1];
    }

    // every lane stores (the three beyond the element write zeros into the
    // padding), so that each wave writes whole lines of its element run
    const uint32_t soff = (uint32_t)(e * SRUN + t) * (uint32_t)sizeof(R);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (MODE == 0) {
            __builtin_nontemporal_store(act ? Rv[v] : (R)0, gptr<R>(P.outs[v], soff));
        } else {
            const R dq = MODE == 1 ? A * dqv[v] + dt * Rv[v] : dt * Rv[v];
            const R yn = o.Yr[v] + B * dq;
            __builtin_nontemporal_store(act ? dq : (R)0, gptr<R>(P.dQs[v], soff));
            __builtin_nontemporal_store(act ? yn : (R)0, gptr<R>(P.outs[v], soff));
            if (MOIST && VISC) Rv[v] = yn;  // keep the output state for its temperature
        }
    }
    if (!act) return;
    if (MOIST && VISC && MODE != 0 && P.Tnext != nullptr) {
        // temperature of the output state, from the input state's as the
        // Newton start: the next stage's passes read it instead of solving
        double qcnew;
        double yn[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if constexpr (sizeof(R) == 8) yn[v] = Rv[v];
            else yn[v] = (double)Rv[v] + (double)o.bg[v];
        }
        const double Tnew = moist_T_guess(yn[0], yn[1], yn[2], yn[3], yn[4], yn[NV - 1], z, P.g, o.T, ICE, qcnew);
        const int64_t nt = (int64_t)e * run_nodes<double>() + t;
        __builtin_nontemporal_store(Tnew, &P.Tnext[nt]);
        __builtin_nontemporal_store(qcnew, &P.Tnext[P.nnT + nt]);
    }
}

// contravariant total flux J a^d . F per (variable, direction); after the
// divergence each face task overwrites its own-node entry with the lift of
// (n.F^- - n.F^*)
#define CM_TEND_LDS                          \
    __shared__ R sG[NV * 3][NP];             \
    __shared__ R sD[NQ * NQ];                \
    __shared__ R sP[tend_keeps_p<R, MOIST, VISC>() ? 4 : 1][BLOCK]; /* u v w c */ \
    __shared__ R sY[NV][BLOCK]; /* own state, for the face tasks */

// one element per block: own loads first, then the first face task's, so
// that their latency overlaps phase A
// VAR: numerical flux of a dry model (0 Rusanov, 1 Roe, 2 HLLC), or for a
// moist model 1 = thermodynamics with the ice phase
template <typename R, bool MOIST, bool WARP, bool VISC, int MODE, int VAR>
__global__ __launch_bounds__(BLOCK) void k_tend(const KParams P, const R* __restrict__ F2, R A, R B, R dt)
{
    constexpr int NV = MOIST ? 6 : 5;
    CM_TEND_LDS
    const int e = elem_of_block(P, blockIdx.x);
    const int t = threadIdx.x;
    const int tt = t < NP ? t : NP - 1;
    const int ex = e % P.ne0, ey = (e / P.ne0) % P.ne1, ez = e / (P.ne0 * P.ne1);
    OwnLoad<R, MOIST, WARP, VISC, MODE> o;
    const R dval = dmat<R>(t < NQ * NQ ? t / NQ : 0, t < NQ * NQ ? t % NQ : 0);
    own_load<R, MOIST, WARP, VISC, MODE>(P, e, ez, tt, o);
    FaceLoad<R, MOIST, WARP, VISC> ft0;
    face_load<R, MOIST, WARP, VISC>(P, F2, t, e, ex, ey, ez, ft0);
    tend_element<R, MOIST, WARP, VISC, MODE, VAR>(P, e, t, o, ft0, dval, sG, sP, sY, sD, F2, A, B, dt);
}

#undef CM_TEND_LDS

// per-variable and per-word bases of one launch's arrays
template <typename R>
static void set_bases(KParams& P, const void* Y, void* out, void* dQ, void* F2)
{
    for (int v = 0; v < 6; ++v) {
        P.Ys[v] = Y ? (const void*)((const R*)Y + v * P.nnS) : nullptr;
        P.outs[v] = out ? (void*)((R*)out + v * P.nnS) : nullptr;
        P.dQs[v] = dQ ? (void*)((R*)dQ + v * P.nnS) : nullptr;
    }
    for (int q = 0; q < 14; ++q) P.F2s[q] = F2 ? (void*)((R*)F2 + q * P.nnf) : nullptr;
}

template <typename R, bool MOIST, bool WARP>
static hipError_t launch_typed(cm_model* m, const void* Y, void* out, void* dQ, int mode, double A, double B,
                               double dt, hipStream_t s)
{
    KParams P = m->kp;
    set_bases<R>(P, Y, out, dQ, m->d_F2);
    const bool moist_visc = MOIST && m->d_T[0] != nullptr;
    if (moist_visc) {
        // stages 2..5 of an LSRK step (mode 1) find their input state's T in
        // d_T[tsel], written by the previous stage's tendency pass
        P.Tn = m->d_T[m->tsel];
        P.Tnext = mode != 0 ? m->d_T[m->tsel ^ 1] : nullptr;
        P.T_given = mode == 1;
    }
    const dim3 grid(P.n_elem), block(BLOCK);
    const R* F2 = (const R*)m->d_F2;
    const bool visc = m->desc.closure != CM_CLOSURE_NONE;
    const bool ice = MOIST && P.ice;
    if (visc) {
        cm_model::ProfRec* r = prof_begin(m, 0, s);
        if (m->desc.closure == CM_CLOSURE_MLP)
            hipLaunchKernelGGL((k_grad<R, MOIST, WARP, true>), grid, block, 0, s, P);
        else if (ice)
            hipLaunchKernelGGL((k_grad<R, MOIST, WARP, false, false, MOIST>), grid, block, 0, s, P);
        else
            hipLaunchKernelGGL((k_grad<R, MOIST, WARP, false>), grid, block, 0, s, P);
        prof_end(r, s);
    }
    cm_model::ProfRec* rt = prof_begin(m, 1, s);
#define CM_TEND(V, MD, FL)                                                                                  \
    hipLaunchKernelGGL((k_tend<R, MOIST, WARP, V, MD, FL>), grid, block, 0, s, P, F2, (R)A, (R)B, (R)dt)
#define CM_TEND_MODES(V, FL)              \
    do {                                  \
        if (mode == 0) CM_TEND(V, 0, FL); \
        else if (mode == 1) CM_TEND(V, 1, FL); \
        else CM_TEND(V, 2, FL);           \
    } while (0)
    // Roe and HLLC are instantiated for dry models only (the model rejects
    // them otherwise); for moist models the same slot selects the ice phase
    const int flux = MOIST ? (ice ? 1 : 0) : m->desc.flux;
    if (visc) {
        if (flux == 1) CM_TEND_MODES(true, 1);
        else if (flux == 2) CM_TEND_MODES(true, MOIST ? 0 : 2);
        else CM_TEND_MODES(true, 0);
    } else {
        if (flux == 1) CM_TEND_MODES(false, 1);
        else if (flux == 2) CM_TEND_MODES(false, MOIST ? 0 : 2);
        else CM_TEND_MODES(false, 0);
    }
#undef CM_TEND_MODES
#undef CM_TEND
    prof_end(rt, s);
    if (moist_visc && mode != 0) m->tsel ^= 1;
    return hipGetLastError();
}

hipError_t launch_grad_only(cm_model* m, const void* Y, hipStream_t s)
{
    KParams P = m->kp;
    set_bases<double>(P, Y, nullptr, nullptr, m->d_F2);
    const bool moist = m->desc.nvar == 6;
    const bool warp = m->grid->desc.topo == 1;
    if (m->desc.precision != CM_FP64) return hipErrorInvalidValue;
    const dim3 grid(P.n_elem), block(BLOCK);
    if (moist) {
        if (warp) hipLaunchKernelGGL((k_grad<double, true, true, false, true>), grid, block, 0, s, P);
        else hipLaunchKernelGGL((k_grad<double, true, false, false, true>), grid, block, 0, s, P);
    } else {
        if (warp) hipLaunchKernelGGL((k_grad<double, false, true, false, true>), grid, block, 0, s, P);
        else hipLaunchKernelGGL((k_grad<double, false, false, false, true>), grid, block, 0, s, P);
    }
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
