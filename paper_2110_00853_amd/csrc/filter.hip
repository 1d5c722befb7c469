// Exponential modal filter (Sect. 5.4, eq. exponential_filter): one element
// per 128-thread block; the deviations from the background of the selected
// variables go through the 1-D filter matrix along xi1, xi2 and xi3 (three
// passes of five-term sums) and the background is added back.  Lane
// (v, a, b) of the 125 works on the five nodes of one line of variable v:
// along xi1 it loads them from memory and leaves the result in LDS, along
// xi2 it filters in LDS, along xi3 it stores to memory (four barriers, the
// first of them with the loads in flight; one state-sized tile of LDS per
// element).
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
    constexpr int MV = 6;
    __shared__ double T[MV][NP];
    __shared__ double sF[NQ * NQ];  // the 1-D matrix (a lane-indexed read of the launch arguments would be a
                                    // vector load at every use)
    const int e = blockIdx.x;
    const int t = threadIdx.x;
    if (t < NQ * NQ) sF[t] = A.F[t];
    // lane t < 125: variable v = t / 25, line (a, b) = (t % 5, (t / 5) % 5);
    // a sixth variable (moist models) takes lanes 0-24 a second time
    const int v0 = t / (NQ * NQ), ab = t % (NQ * NQ);
    const int a = ab % NQ, b = ab / NQ;
    const int nv = A.nvar;
    const int64_t base = (int64_t)e * SRUN;
    const int ez = e / A.ne01;
    // the background of node n of this element for variable v (FP32-bulk
    // states hold the deviation from it already)
    auto ref = [&](int v, int n) -> double {
        if (sizeof(R) != 8) return 0.0;
        const int64_t ri = A.ref_per_node ? (int64_t)e * NP + n : (int64_t)ez * NQ + n / (NQ * NQ);
        return A.Yref[v * A.nref + ri];
    };
    // xi1: line (j, k) = (a, b), nodes i + 5 a + 25 b; the loads go out
    // before the barrier that publishes the matrix
    double x1[2][NQ];
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        const int v = pass == 0 ? v0 : 5;
        const bool on = (pass == 0 ? t < 5 * NQ * NQ : t < NQ * NQ) && v < nv && ((A.mask >> v) & 1);
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const int n = i + NQ * (a + NQ * b);
            x1[pass][i] = on ? (double)Y[v * A.nnS + base + n] - ref(v, n) : 0.0;
        }
    }
    __syncthreads();
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        const int v = pass == 0 ? v0 : 5;
        const bool on = (pass == 0 ? t < 5 * NQ * NQ : t < NQ * NQ) && v < nv && ((A.mask >> v) & 1);
        if (on) {
#pragma unroll
            for (int i = 0; i < NQ; ++i) {
                double s = 0.0;
#pragma unroll
                for (int l = 0; l < NQ; ++l) s += sF[i * NQ + l] * x1[pass][l];
                T[v][i + NQ * (a + NQ * b)] = s;
            }
        }
    }
    __syncthreads();
    // xi2: line (i, k) = (a, b), nodes a + 5 j + 25 b
    double y[2][NQ];
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        const int v = pass == 0 ? v0 : 5;
        const bool on = (pass == 0 ? t < 5 * NQ * NQ : t < NQ * NQ) && v < nv && ((A.mask >> v) & 1);
        if (on) {
            double x[NQ];
#pragma unroll
            for (int j = 0; j < NQ; ++j) x[j] = T[v][a + NQ * (j + NQ * b)];
#pragma unroll
            for (int j = 0; j < NQ; ++j) {
                double s = 0.0;
#pragma unroll
                for (int l = 0; l < NQ; ++l) s += sF[j * NQ + l] * x[l];
                y[pass][j] = s;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        const int v = pass == 0 ? v0 : 5;
        const bool on = (pass == 0 ? t < 5 * NQ * NQ : t < NQ * NQ) && v < nv && ((A.mask >> v) & 1);
        if (on) {
#pragma unroll
            for (int j = 0; j < NQ; ++j) T[v][a + NQ * (j + NQ * b)] = y[pass][j];
        }
    }
    __syncthreads();
    // xi3: line (i, j) = (a, b), nodes a + 5 b + 25 k
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        const int v = pass == 0 ? v0 : 5;
        const bool on = (pass == 0 ? t < 5 * NQ * NQ : t < NQ * NQ) && v < nv && ((A.mask >> v) & 1);
        if (on) {
            double x[NQ];
#pragma unroll
            for (int k = 0; k < NQ; ++k) x[k] = T[v][a + NQ * (b + NQ * k)];
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                double s = 0.0;
#pragma unroll
                for (int l = 0; l < NQ; ++l) s += sF[k * NQ + l] * x[l];
                const int n = a + NQ * (b + NQ * k);
                Y[v * A.nnS + base + n] = (R)(ref(v, n) + s);
            }
        }
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
