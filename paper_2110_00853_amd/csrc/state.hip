// Conversion between full FP64 states and a model's stored states.  FP64
// models store full values; FP32-bulk models store d = float(Y - Y_bg), the
// deviation from the background as given (FP64), so that the rounding error
// of the stored state scales with the deviation rather than with the
// hydrostatic background.  The kernels evolve d about the background rounded
// to float (B, with the reference pressure and density computed from B, so
// that d = 0 is exactly at rest); export returns Y_bg + d, so that export
// and import invert each other.  Both sides use the padded layout
// [nvar][n_elem x SRUN]; padding slots are written as zero.
#include "cm_impl.hpp"

namespace cm {

struct ConvArgs {
    int nvar, ne01, ref_per_node;
    int64_t nnS, nref, n_slots;
    const double* bg64;  // the background as given; null: full values
};

__device__ __forceinline__ double conv_bg(const ConvArgs& A, int v, int64_t q)
{
    if (!A.bg64) return 0.0;
    const int64_t e = q / SRUN;
    const int t = (int)(q % SRUN);
    const int64_t ri = A.ref_per_node ? e * NP + t : (e / A.ne01) * NQ + t / (NQ * NQ);
    return A.bg64[v * A.nref + ri];
}

// full FP64 -> stored (type R)
template <typename R>
__global__ __launch_bounds__(256) void k_import(const ConvArgs A, const double* __restrict__ Y, R* __restrict__ S)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= A.n_slots) return;
    const bool node = (int)(q % SRUN) < NP;
    for (int v = 0; v < A.nvar; ++v)
        S[v * A.nnS + q] = node ? (R)(Y[v * A.nnS + q] - conv_bg(A, v, q)) : (R)0;
}

// stored (type R) -> full FP64
template <typename R>
__global__ __launch_bounds__(256) void k_export(const ConvArgs A, const R* __restrict__ S, double* __restrict__ Y)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= A.n_slots) return;
    const bool node = (int)(q % SRUN) < NP;
    for (int v = 0; v < A.nvar; ++v)
        Y[v * A.nnS + q] = node ? (double)S[v * A.nnS + q] + conv_bg(A, v, q) : 0.0;
}

hipError_t launch_state_convert(const cm_model* m, const void* src, void* dst, bool to_storage, hipStream_t s)
{
    ConvArgs A;
    A.nvar = m->desc.nvar;
    A.ne01 = m->grid->desc.ne[0] * m->grid->desc.ne[1];
    A.ref_per_node = m->ref_per_node;
    A.nnS = m->grid->n_elem * SRUN;
    A.n_slots = A.nnS;
    A.nref = m->nref;
    A.bg64 = m->desc.precision == CM_FP32_BULK ? m->d_bg64 : nullptr;
    const dim3 grid((unsigned)((A.n_slots + 255) / 256)), block(256);
    if (m->desc.precision == CM_FP64) {
        if (to_storage) hipLaunchKernelGGL(k_import<double>, grid, block, 0, s, A, (const double*)src, (double*)dst);
        else hipLaunchKernelGGL(k_export<double>, grid, block, 0, s, A, (const double*)src, (double*)dst);
    } else {
        if (to_storage) hipLaunchKernelGGL(k_import<float>, grid, block, 0, s, A, (const double*)src, (float*)dst);
        else hipLaunchKernelGGL(k_export<float>, grid, block, 0, s, A, (const float*)src, (double*)dst);
    }
    return hipGetLastError();
}

}  // namespace cm
