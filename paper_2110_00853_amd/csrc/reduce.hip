// Conservation and health diagnostics (Sect. 6: normalised mass and total
// energy integrals).  Deterministic two-stage reduction: a fixed node->thread
// assignment with Neumaier-compensated FP64 sums per thread, a fixed-order
// tree per block, and one block combining the per-block partials in order.
#include <cmath>
#include <mutex>

#include "cm_impl.hpp"
#include "thermo.hpp"

namespace cm {

constexpr int RB = 256;      // threads per reduction block
constexpr int NPART = 16;    // doubles per partial record

struct Neu {
    double s, c;
};

__device__ __forceinline__ void neu_add(Neu& a, double x)
{
    const double t = a.s + x;
    if (fabs(a.s) >= fabs(x)) a.c += (a.s - t) + x;
    else a.c += (x - t) + a.s;
    a.s = t;
}

__device__ __forceinline__ void neu_merge(Neu& a, const Neu& b)
{
    neu_add(a, b.s);
    a.c += b.c;
}

// temperature and sound speed of one node (the thermodynamics of the passes)
template <bool MOIST>
__device__ void temp_sound(double rho, double mx, double my, double mz, double re, double rq, double z, double g,
                           bool ice, double& T, double& c)
{
    Th o;
    thermo<MOIST>(rho, mx, my, mz, re, rq, z, g, ice, o);
    T = o.T;
    c = o.c;
}

struct DiagArgs {
    int64_t nn;
    int64_t nnS;             // state stride (n_elem x SRUN slots per variable)
    int ne0, ne1;
    double lo2, h2, zg[NQ];
    double w[NQ];
    double Jc;               // Cartesian Jacobian
    const double* invJ;      // warped: per-node 1/J (FP64) or null
    const double* zn;        // warped: node heights or null
    double g, dt, dmin;
    int ice;
    // FP32-bulk states hold deviations from this background (null: full values)
    const float* bg32;
    int64_t nref;
    int ref_per_node;
};

template <typename R, bool MOIST>
__global__ __launch_bounds__(RB) void k_diag1(const DiagArgs A, const R* __restrict__ Y, double* __restrict__ part)
{
    constexpr int NV = MOIST ? 6 : 5;
    Neu acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    double maxw = 0.0, maxcfl = 0.0, Tmin = INFINITY, Tmax = -INFINITY, nonfin = 0.0;
    const int64_t stride = (int64_t)gridDim.x * RB;
    for (int64_t n = (int64_t)blockIdx.x * RB + threadIdx.x; n < A.nn; n += stride) {
        const int t = (int)(n % NP);
        const int64_t e = n / NP;
        const int64_t slot = e * SRUN + t;  // the node's slot in the state buffer
        double y[NV];
        bool fin = true;
        const int i = t % NQ, j = (t / NQ) % NQ, k = t / (NQ * NQ);
        const int64_t ri = A.ref_per_node ? n : (e / ((int64_t)A.ne0 * A.ne1)) * NQ + k;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            y[v] = (double)Y[v * A.nnS + slot] + (A.bg32 ? (double)A.bg32[v * A.nref + ri] : 0.0);
            if (!isfinite(y[v])) { nonfin += 1.0; fin = false; }
        }
        if (!fin) continue;
        const double J = A.invJ ? 1.0 / A.invJ[n] : A.Jc;
        const double wJ = A.w[i] * A.w[j] * A.w[k] * J;
        const double z = A.zn ? A.zn[n] : A.lo2 + ((double)(e / ((int64_t)A.ne0 * A.ne1)) + A.zg[k]) * A.h2;
        neu_add(acc[0], wJ * y[0]);
        neu_add(acc[1], wJ * y[4]);
        if (MOIST) neu_add(acc[2], wJ * y[5]);
        neu_add(acc[3], wJ * 0.5 * (y[1] * y[1] + y[2] * y[2] + y[3] * y[3]) / y[0]);
        const double ir = 1.0 / y[0];
        const double aw = fabs(y[3] * ir);
        maxw = aw > maxw ? aw : maxw;
        double T, c;
        temp_sound<MOIST>(y[0], y[1], y[2], y[3], y[4], MOIST ? y[5] : 0.0, z, A.g, A.ice != 0, T, c);
        Tmin = T < Tmin ? T : Tmin;
        Tmax = T > Tmax ? T : Tmax;
        if (A.dt > 0.0) {
            const double sp = sqrt(y[1] * y[1] + y[2] * y[2] + y[3] * y[3]) * ir + c;
            const double cfl = sp * A.dt / A.dmin;
            maxcfl = cfl > maxcfl ? cfl : maxcfl;
        }
    }
    __shared__ double sh[RB][NPART];
    const int tid = threadIdx.x;
    for (int q = 0; q < 4; ++q) { sh[tid][2 * q] = acc[q].s; sh[tid][2 * q + 1] = acc[q].c; }
    sh[tid][8] = maxw; sh[tid][9] = maxcfl; sh[tid][10] = Tmin; sh[tid][11] = Tmax; sh[tid][12] = nonfin;
    __syncthreads();
    for (int off = RB / 2; off > 0; off >>= 1) {
        if (tid < off) {
            for (int q = 0; q < 4; ++q) {
                Neu a = {sh[tid][2 * q], sh[tid][2 * q + 1]};
                const Neu b = {sh[tid + off][2 * q], sh[tid + off][2 * q + 1]};
                neu_merge(a, b);
                sh[tid][2 * q] = a.s;
                sh[tid][2 * q + 1] = a.c;
            }
            sh[tid][8] = fmax(sh[tid][8], sh[tid + off][8]);
            sh[tid][9] = fmax(sh[tid][9], sh[tid + off][9]);
            sh[tid][10] = fmin(sh[tid][10], sh[tid + off][10]);
            sh[tid][11] = fmax(sh[tid][11], sh[tid + off][11]);
            sh[tid][12] = sh[tid][12] + sh[tid + off][12];
        }
        __syncthreads();
    }
    if (tid < NPART) part[(int64_t)blockIdx.x * NPART + tid] = tid < 13 ? sh[0][tid] : 0.0;
}

// combine the per-block partials in block order (one thread, deterministic)
// combine of the per-block partials: each thread merges a strided subset
// (compensated sums, extrema), then a fixed pairwise tree in LDS, so the
// result does not depend on timing
__global__ __launch_bounds__(RB) void k_diag2(const double* __restrict__ part, int nblk, double* __restrict__ out)
{
    __shared__ double sh[RB][NPART];
    const int tid = threadIdx.x;
    Neu acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    double maxw = 0.0, maxcfl = 0.0, Tmin = INFINITY, Tmax = -INFINITY, nonfin = 0.0;
    for (int b = tid; b < nblk; b += RB) {
        const double* p = part + (int64_t)b * NPART;
        for (int q = 0; q < 4; ++q) neu_merge(acc[q], Neu{p[2 * q], p[2 * q + 1]});
        maxw = fmax(maxw, p[8]);
        maxcfl = fmax(maxcfl, p[9]);
        Tmin = fmin(Tmin, p[10]);
        Tmax = fmax(Tmax, p[11]);
        nonfin += p[12];
    }
    for (int q = 0; q < 4; ++q) { sh[tid][2 * q] = acc[q].s; sh[tid][2 * q + 1] = acc[q].c; }
    sh[tid][8] = maxw; sh[tid][9] = maxcfl; sh[tid][10] = Tmin; sh[tid][11] = Tmax; sh[tid][12] = nonfin;
    __syncthreads();
    for (int half = RB / 2; half > 0; half >>= 1) {
        if (tid < half) {
            const double* o = sh[tid + half];
            for (int q = 0; q < 4; ++q) {
                Neu a{sh[tid][2 * q], sh[tid][2 * q + 1]};
                neu_merge(a, Neu{o[2 * q], o[2 * q + 1]});
                sh[tid][2 * q] = a.s;
                sh[tid][2 * q + 1] = a.c;
            }
            sh[tid][8] = fmax(sh[tid][8], o[8]);
            sh[tid][9] = fmax(sh[tid][9], o[9]);
            sh[tid][10] = fmin(sh[tid][10], o[10]);
            sh[tid][11] = fmax(sh[tid][11], o[11]);
            sh[tid][12] += o[12];
        }
        __syncthreads();
    }
    if (tid == 0) {
        for (int q = 0; q < 4; ++q) out[q] = sh[0][2 * q] + sh[0][2 * q + 1];
        for (int q = 4; q < 9; ++q) out[q] = sh[0][q + 4];
    }
}

// both passes over a workspace of n_records partial records (16 doubles
// each): the first n_records - 1 hold the per-block partials, the last one
// the combined result.  The first pass strides over the nodes, so any grid
// fits; the block count, and with it the order of the compensated sums,
// depends only on the node count and n_records.
static hipError_t diagnostics_ws(const cm_model* m, const void* Y, double dt, cm_diag* outp, hipStream_t s,
                                 double* ws, int n_records)
{
    const cm_grid* g = m->grid;
    DiagArgs A;
    A.nn = g->n_nodes;
    A.nnS = g->n_elem * SRUN;
    A.ne0 = g->desc.ne[0];
    A.ne1 = g->desc.ne[1];
    A.lo2 = g->desc.lo[2];
    A.h2 = g->h[2];
    for (int q = 0; q < NQ; ++q) { A.zg[q] = 0.5 * (1.0 + g->xi[q]); A.w[q] = g->w[q]; }
    A.Jc = 0.125 * g->h[0] * g->h[1] * g->h[2];
    A.invJ = g->d_metrics64 ? g->d_metrics64 + 9 * g->n_nodes : nullptr;
    A.zn = g->d_z;
    A.g = m->desc.g;
    A.ice = m->desc.ice;
    A.dt = dt;
    A.dmin = g->dmin;
    A.bg32 = m->d_bg32;
    A.nref = m->nref;
    A.ref_per_node = m->ref_per_node;
    int nblk = (int)((A.nn + RB - 1) / RB);
    if (nblk > n_records - 1) nblk = n_records - 1;
    double* part = ws;
    double* dout = ws + (int64_t)(n_records - 1) * NPART;
    const bool moist = m->desc.nvar == 6;
    if (m->desc.precision == CM_FP64) {
        if (moist) hipLaunchKernelGGL((k_diag1<double, true>), dim3(nblk), dim3(RB), 0, s, A, (const double*)Y, part);
        else hipLaunchKernelGGL((k_diag1<double, false>), dim3(nblk), dim3(RB), 0, s, A, (const double*)Y, part);
    } else {
        if (moist) hipLaunchKernelGGL((k_diag1<float, true>), dim3(nblk), dim3(RB), 0, s, A, (const float*)Y, part);
        else hipLaunchKernelGGL((k_diag1<float, false>), dim3(nblk), dim3(RB), 0, s, A, (const float*)Y, part);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag2, dim3(1), dim3(RB), 0, s, part, nblk, dout);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    double h[9];
    e = hipMemcpyAsync(h, dout, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    outp->mass = h[0];
    outp->energy = h[1];
    outp->water = h[2];
    outp->ke = h[3];
    outp->max_abs_w = h[4];
    outp->max_cfl = h[5];
    outp->T_min = h[6];
    outp->T_max = h[7];
    outp->n_nonfinite = (int64_t)h[8];
    return hipSuccess;
}

hipError_t launch_diagnostics(const cm_model* m, const void* Y, double dt, cm_diag* outp, hipStream_t s)
{
    return diagnostics_ws(m, Y, dt, outp, s, m->d_partials, m->n_partials);
}

// Workspace of the allocation-free diagnostics: DIAG_SCRATCH_RECORDS partial
// records in a file-scope device array (256 KiB; every device the library
// runs on holds its own copy until the process ends).  Host code never
// passes the array's name to a kernel: its device address, per device,
// comes from hipGetSymbolAddress on the first call on that device.
static __device__ __align__(256) double scratch[DIAG_SCRATCH_RECORDS * NPART];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t diag_scratch_address(int device, double** out)
{
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        // the caller has made `device` current
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = (double*)p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

hipError_t launch_diagnostics_static(const cm_model* m, const void* Y, double dt, cm_diag* outp, hipStream_t s)
{
    double* ws = nullptr;
    const hipError_t e = diag_scratch_address(m->grid->device, &ws);
    if (e != hipSuccess) return e;
    return diagnostics_ws(m, Y, dt, outp, s, ws, DIAG_SCRATCH_RECORDS);
}

}  // namespace cm
