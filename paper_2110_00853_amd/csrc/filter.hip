// Exponential modal filter (Sect. 5.4, eq. exponential_filter): one element
// per 128-thread block; the deviations from the background of all selected
// variables go together through the 1-D filter matrix along xi1, xi2 and
// xi3 in LDS (three passes of five-term sums, four barriers per element) and
// the background is added back.
// Elements are independent, so the state is filtered in place.
#include "cm_impl.hpp"

namespace cm {

struct FilterArgs {
    double F[NQ * NQ];       // F[i][l]: node i from node l along one direction
    int mask, nvar, ref_per_node, ne01;
    int64_t nnS;             // state stride
    int64_t nref;            // background entries per variable
    const double* Yref;      // [nvar][nref]
};

template <typename R>
__global__ __launch_bounds__(BLOCK) void k_filter(const FilterArgs A, R* __restrict__ Y)
{
    constexpr int MV = 6;  // at most six variables, filtered together
    __shared__ double a[MV][BLOCK], b[MV][BLOCK];
    __shared__ double sF[NQ * NQ];  // the 1-D matrix (a lane-indexed read of the launch arguments would be a
                                    // vector load at every use)
    const int e = blockIdx.x;
    const int t = threadIdx.x;
    if (t < NQ * NQ) sF[t] = A.F[t];
    const bool act = t < NP;
    const int tt = act ? t : NP - 1;
    const int i = tt % NQ, j = (tt / NQ) % NQ, k = tt / (NQ * NQ);
    const int64_t ri = A.ref_per_node ? (int64_t)e * NP + tt : (int64_t)(e / A.ne01) * NQ + k;
    // every selected variable's loads first, so that their latencies overlap
    double ref[MV];
#pragma unroll
    for (int v = 0; v < MV; ++v) {
        if (v >= A.nvar || !((A.mask >> v) & 1)) continue;
        // FP32-bulk states already hold the deviation from the background
        ref[v] = sizeof(R) == 8 ? A.Yref[v * A.nref + ri] : 0.0;
        const double yv = act ? (double)Y[v * A.nnS + (int64_t)e * SRUN + tt] : 0.0;
        a[v][t] = act ? yv - ref[v] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < MV; ++v) {
        if (v >= A.nvar || !((A.mask >> v) & 1)) continue;
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < NQ; ++l) s += sF[i * NQ + l] * a[v][l + NQ * (j + NQ * k)];
        b[v][t] = s;
    }
    __syncthreads();
    double s2[MV];
#pragma unroll
    for (int v = 0; v < MV; ++v) {
        if (v >= A.nvar || !((A.mask >> v) & 1)) continue;
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < NQ; ++l) s += sF[j * NQ + l] * b[v][i + NQ * (l + NQ * k)];
        s2[v] = s;
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < MV; ++v)
        if (v < A.nvar && ((A.mask >> v) & 1)) a[v][t] = s2[v];
    __syncthreads();
#pragma unroll
    for (int v = 0; v < MV; ++v) {
        if (v >= A.nvar || !((A.mask >> v) & 1)) continue;
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < NQ; ++l) s += sF[k * NQ + l] * a[v][i + NQ * (j + NQ * l)];
        if (act) Y[v * A.nnS + (int64_t)e * SRUN + tt] = (R)(ref[v] + s);
    }
}

hipError_t launch_exp_filter(const cm_model* m, void* Y, int mask, const double* F1, hipStream_t s)
{
    FilterArgs A;
    for (int q = 0; q < NQ * NQ; ++q) A.F[q] = F1[q];
    A.mask = mask;
    A.nvar = m->desc.nvar;
    A.ref_per_node = m->ref_per_node;
    A.ne01 = m->grid->desc.ne[0] * m->grid->desc.ne[1];
    A.nnS = m->grid->n_elem * SRUN;
    A.nref = m->ref_per_node ? m->grid->n_nodes : (int64_t)m->grid->desc.ne[2] * NQ;
    A.Yref = m->d_Yref;
    const dim3 grid((unsigned)m->grid->n_elem), block(BLOCK);
    if (m->desc.precision == CM_FP64)
        hipLaunchKernelGGL(k_filter<double>, grid, block, 0, s, A, (double*)Y);
    else
        hipLaunchKernelGGL(k_filter<float>, grid, block, 0, s, A, (float*)Y);
    return hipGetLastError();
}

}  // namespace cm
