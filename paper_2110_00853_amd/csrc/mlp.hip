// Learned SGS closure: network object, BF16-MFMA training kernels (forward,
// backward, Adam) and the weights of the fused closure inference.
//
// Training works on batches of standardised inputs X [n][12] and targets
// T [n][2] for the raw network outputs.  Every matrix product is a
// 16x16x16 bf16 MFMA tile loop with FP32 accumulation; master weights, Adam
// moments and activations are FP32.  Loss: (1/n) sum |O - T|^2.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "cm_impl.hpp"
#include "mlp_common.hpp"

namespace cm {

struct GemmArgs {
    int M, N, K;
    const float* A;
    int64_t a_rs, a_cs;   // A(i, k) = A[i a_rs + k a_cs]
    const float* B;
    int64_t b_rs, b_cs;   // B(k, j) = B[k b_rs + j b_cs]
    float* C;
    int64_t ldc;          // C(i, j) = C[i ldc + j]
    const float* bias;    // optional, per column
    const float* dz;      // optional: C(i, j) *= silu'(dz[i ldc + j])
    float* H;             // optional: H(i, j) = silu(C(i, j))
};

// one 16 x 16 output tile per wave, 4 waves per block
__global__ __launch_bounds__(256) void k_gemm(const GemmArgs g)
{
    const int lane = threadIdx.x & 63;
    const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int tn = (g.N + 15) / 16, tm = (g.M + 15) / 16;
    if (wid >= tm * tn) return;
    const int m0 = (wid / tn) * 16, n0 = (wid % tn) * 16;
    const int r = lane & 15, kq = (lane >> 4) * 4;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    const bool row_ok = m0 + r < g.M, col_ok = n0 + r < g.N;
    for (int k0 = 0; k0 < g.K; k0 += 16) {
        bf16x4 a, b;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = k0 + kq + q;
            const float av = (row_ok && k < g.K) ? g.A[(int64_t)(m0 + r) * g.a_rs + (int64_t)k * g.a_cs] : 0.0f;
            const float bv = (col_ok && k < g.K) ? g.B[(int64_t)k * g.b_rs + (int64_t)(n0 + r) * g.b_cs] : 0.0f;
            a[q] = (short)f2bf(av);
            b[q] = (short)f2bf(bv);
        }
        acc = mfma16(a, b, acc);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = m0 + kq + q, j = n0 + r;
        if (i < g.M && j < g.N) {
            float c = acc[q] + (g.bias ? g.bias[j] : 0.0f);
            const int64_t o = (int64_t)i * g.ldc + j;
            if (g.dz) c *= dsilu_f(g.dz[o]);
            g.C[o] = c;
            if (g.H) g.H[o] = silu_f(c);
        }
    }
}

static hipError_t gemm(const GemmArgs& g, hipStream_t s)
{
    const int tiles = ((g.M + 15) / 16) * ((g.N + 15) / 16);
    hipLaunchKernelGGL(k_gemm, dim3((tiles + 3) / 4), dim3(256), 0, s, g);
    return hipGetLastError();
}

// dO = 2 (O - T) / n and per-block sums of squared residuals
__global__ __launch_bounds__(256) void k_mse(int n, const float* __restrict__ O, const float* __restrict__ T,
                                             float* __restrict__ dO, float* __restrict__ part)
{
    __shared__ float sh[256];
    float acc = 0.0f;
    for (int q = blockIdx.x * 256 + threadIdx.x; q < 2 * n; q += gridDim.x * 256) {
        const float r = O[q] - T[q];
        dO[q] = 2.0f * r / (float)n;
        acc += r * r;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// out[j] = sum_i D[i ld + j] (bias gradients), one block per column
__global__ __launch_bounds__(256) void k_colsum(int M, int N, const float* __restrict__ D, int64_t ld,
                                                float* __restrict__ out)
{
    __shared__ float sh[256];
    const int j = blockIdx.x;
    if (j >= N) return;
    float acc = 0.0f;
    for (int i = threadIdx.x; i < M; i += 256) acc += D[(int64_t)i * ld + j];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = sh[0];
}

// Adam with bias correction (Kingma & Ba); c1 = 1 - b1^t, c2 = 1 - b2^t
__global__ void k_adam(int n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.0f - b1) * gq;
    const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

}  // namespace cm

struct cm_mlp {
    int device = 0;
    cm_mlp_desc desc{};
    float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    int step = 0;
    int cap = 0;
    float *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *Z3 = nullptr, *H3 = nullptr;
    float *O = nullptr, *dO = nullptr, *dZ3 = nullptr, *dZ2 = nullptr, *dZ1 = nullptr, *part = nullptr;
};

using namespace cm;

namespace {

void free_acts(cm_mlp* n)
{
    float** bufs[] = {&n->Z1, &n->H1, &n->Z2, &n->H2, &n->Z3, &n->H3, &n->O, &n->dO, &n->dZ3, &n->dZ2, &n->dZ1, &n->part};
    for (float** b : bufs) {
        if (*b) (void)hipFree(*b);
        *b = nullptr;
    }
    n->cap = 0;
}

hipError_t ensure_capacity(cm_mlp* n, int batch)
{
    if (batch <= n->cap) return hipSuccess;
    free_acts(n);
    const size_t h = sizeof(float) * (size_t)batch * MLP_NH;
    hipError_t e = hipSuccess;
    float** hb[] = {&n->Z1, &n->H1, &n->Z2, &n->H2, &n->Z3, &n->H3, &n->dZ3, &n->dZ2, &n->dZ1};
    for (float** b : hb)
        if (e == hipSuccess) e = hipMalloc(b, h);
    if (e == hipSuccess) e = hipMalloc(&n->O, sizeof(float) * (size_t)batch * MLP_NO);
    if (e == hipSuccess) e = hipMalloc(&n->dO, sizeof(float) * (size_t)batch * MLP_NO);
    if (e == hipSuccess) e = hipMalloc(&n->part, sizeof(float) * 1024);
    if (e == hipSuccess) n->cap = batch;
    return e;
}

GemmArgs ga(int M, int N, int K, const float* A, int64_t ars, int64_t acs, const float* B, int64_t brs, int64_t bcs,
            float* C, int64_t ldc, const float* bias = nullptr, const float* dz = nullptr, float* H = nullptr)
{
    GemmArgs g;
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.a_rs = ars; g.a_cs = acs;
    g.B = B; g.b_rs = brs; g.b_cs = bcs;
    g.C = C; g.ldc = ldc;
    g.bias = bias; g.dz = dz; g.H = H;
    return g;
}

// forward pass storing activations; O = raw outputs [n][2]
hipError_t forward(cm_mlp* net, const float* X, int n, float* O, hipStream_t s)
{
    const float* P = net->p;
    hipError_t e = gemm(ga(n, MLP_NH, MLP_NI, X, MLP_NI, 1, P + OFF_W1, 1, MLP_NI, net->Z1, MLP_NH, P + OFF_B1,
                           nullptr, net->H1), s);
    if (e == hipSuccess)
        e = gemm(ga(n, MLP_NH, MLP_NH, net->H1, MLP_NH, 1, P + OFF_W2, 1, MLP_NH, net->Z2, MLP_NH, P + OFF_B2, nullptr,
                    net->H2), s);
    if (e == hipSuccess)
        e = gemm(ga(n, MLP_NH, MLP_NH, net->H2, MLP_NH, 1, P + OFF_W3, 1, MLP_NH, net->Z3, MLP_NH, P + OFF_B3, nullptr,
                    net->H3), s);
    if (e == hipSuccess)
        e = gemm(ga(n, MLP_NO, MLP_NH, net->H3, MLP_NH, 1, P + OFF_W4, 1, MLP_NH, O, MLP_NO, P + OFF_B4), s);
    return e;
}

// loss gradient into net->g (after forward into net->O); partial loss sums
// into net->part[0 .. nblk)
hipError_t backward(cm_mlp* net, const float* X, const float* T, int n, int* nblk_out, hipStream_t s)
{
    const float* P = net->p;
    float* G = net->g;
    int nblk = (2 * n + 255) / 256;
    if (nblk > 1024) nblk = 1024;
    *nblk_out = nblk;
    hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(256), 0, s, n, net->O, T, net->dO, net->part);
    hipError_t e = hipGetLastError();
    // layer 4
    if (e == hipSuccess) e = gemm(ga(MLP_NO, MLP_NH, n, net->dO, 1, MLP_NO, net->H3, MLP_NH, 1, G + OFF_W4, MLP_NH), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_colsum, dim3(MLP_NO), dim3(256), 0, s, n, MLP_NO, net->dO, (int64_t)MLP_NO, G + OFF_B4);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = gemm(ga(n, MLP_NH, MLP_NO, net->dO, MLP_NO, 1, P + OFF_W4, MLP_NH, 1, net->dZ3, MLP_NH, nullptr, net->Z3), s);
    // layer 3
    if (e == hipSuccess) e = gemm(ga(MLP_NH, MLP_NH, n, net->dZ3, 1, MLP_NH, net->H2, MLP_NH, 1, G + OFF_W3, MLP_NH), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_colsum, dim3(MLP_NH), dim3(256), 0, s, n, MLP_NH, net->dZ3, (int64_t)MLP_NH, G + OFF_B3);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = gemm(ga(n, MLP_NH, MLP_NH, net->dZ3, MLP_NH, 1, P + OFF_W3, MLP_NH, 1, net->dZ2, MLP_NH, nullptr, net->Z2), s);
    // layer 2
    if (e == hipSuccess) e = gemm(ga(MLP_NH, MLP_NH, n, net->dZ2, 1, MLP_NH, net->H1, MLP_NH, 1, G + OFF_W2, MLP_NH), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_colsum, dim3(MLP_NH), dim3(256), 0, s, n, MLP_NH, net->dZ2, (int64_t)MLP_NH, G + OFF_B2);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = gemm(ga(n, MLP_NH, MLP_NH, net->dZ2, MLP_NH, 1, P + OFF_W2, MLP_NH, 1, net->dZ1, MLP_NH, nullptr, net->Z1), s);
    // layer 1
    if (e == hipSuccess) e = gemm(ga(MLP_NH, MLP_NI, n, net->dZ1, 1, MLP_NH, X, MLP_NI, 1, G + OFF_W1, MLP_NI), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_colsum, dim3(MLP_NH), dim3(256), 0, s, n, MLP_NH, net->dZ1, (int64_t)MLP_NH, G + OFF_B1);
        e = hipGetLastError();
    }
    return e;
}

uint64_t splitmix64(uint64_t& x)
{
    uint64_t z = (x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

cm_status check_net(const cm_mlp* n, const char* where)
{
    if (!n) {
        set_error(std::string(where) + ": null network");
        return CM_ERR_ARG;
    }
    return CM_OK;
}

}  // namespace

#define CM_TRY_HIP(expr, where)                           \
    do {                                                  \
        hipError_t _e = (expr);                           \
        if (_e != hipSuccess) return hip_fail(_e, where); \
    } while (0)

extern "C" {

cm_status cm_mlp_create(const cm_mlp_desc* d, uint64_t seed, int hip_device, cm_mlp** out)
{
    if (!d || !out) { set_error("cm_mlp_create: null argument"); return CM_ERR_ARG; }
    *out = nullptr;
    if (d->n_in != MLP_NI || d->n_hidden != MLP_NH || d->n_layers_hidden != 3 || d->n_out != MLP_NO) {
        set_error("cm_mlp_create: only the 12-64-64-64-2 network is supported");
        return CM_ERR_UNSUPPORTED;
    }
    if (!(d->lr > 0.0f) || !(d->beta1 >= 0.0f && d->beta1 < 1.0f) || !(d->beta2 >= 0.0f && d->beta2 < 1.0f) ||
        !(d->eps > 0.0f)) {
        set_error("cm_mlp_create: bad Adam hyper-parameters");
        return CM_ERR_ARG;
    }
    CM_TRY_HIP(hipSetDevice(hip_device), "hipSetDevice");
    cm_mlp* n = new (std::nothrow) cm_mlp();
    if (!n) { set_error("cm_mlp_create: out of host memory"); return CM_ERR_ALLOC; }
    n->device = hip_device;
    n->desc = *d;
    std::vector<float> p(MLP_NPARAM, 0.0f);
    uint64_t st = seed;
    auto uni = [&](float a) { return (float)(((splitmix64(st) >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0) * a; };
    const int offW[4] = {OFF_W1, OFF_W2, OFF_W3, OFF_W4};
    const int fan[4] = {MLP_NI, MLP_NH, MLP_NH, MLP_NH};
    const int nw[4] = {MLP_NH * MLP_NI, MLP_NH * MLP_NH, MLP_NH * MLP_NH, MLP_NO * MLP_NH};
    for (int l = 0; l < 4; ++l)
        for (int q = 0; q < nw[l]; ++q) p[offW[l] + q] = uni(1.0f / std::sqrt((float)fan[l]));
    const size_t bytes = sizeof(float) * MLP_NPARAM;
    hipError_t e = hipMalloc(&n->p, bytes);
    if (e == hipSuccess) e = hipMalloc(&n->m, bytes);
    if (e == hipSuccess) e = hipMalloc(&n->v, bytes);
    if (e == hipSuccess) e = hipMalloc(&n->g, bytes);
    if (e == hipSuccess) e = hipMemcpy(n->p, p.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(n->m, 0, bytes);
    if (e == hipSuccess) e = hipMemset(n->v, 0, bytes);
    if (e != hipSuccess) {
        cm_status s = hip_fail(e, "cm_mlp_create");
        cm_mlp_destroy(n);
        return s;
    }
    *out = n;
    return CM_OK;
}

cm_status cm_mlp_destroy(cm_mlp* n)
{
    if (!n) return CM_OK;
    (void)hipSetDevice(n->device);
    free_acts(n);
    float* b[] = {n->p, n->m, n->v, n->g};
    for (float* q : b)
        if (q) (void)hipFree(q);
    delete n;
    return CM_OK;
}

cm_status cm_mlp_get_params(const cm_mlp* n, float* host)
{
    cm_status st = check_net(n, "cm_mlp_get_params");
    if (st != CM_OK) return st;
    if (!host) { set_error("cm_mlp_get_params: null output"); return CM_ERR_ARG; }
    CM_TRY_HIP(hipSetDevice(n->device), "hipSetDevice");
    CM_TRY_HIP(hipMemcpy(host, n->p, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost), "cm_mlp_get_params");
    return CM_OK;
}

cm_status cm_mlp_set_params(cm_mlp* n, const float* host)
{
    cm_status st = check_net(n, "cm_mlp_set_params");
    if (st != CM_OK) return st;
    if (!host) { set_error("cm_mlp_set_params: null input"); return CM_ERR_ARG; }
    CM_TRY_HIP(hipSetDevice(n->device), "hipSetDevice");
    CM_TRY_HIP(hipMemcpy(n->p, host, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice), "cm_mlp_set_params");
    CM_TRY_HIP(hipMemset(n->m, 0, sizeof(float) * MLP_NPARAM), "cm_mlp_set_params");
    CM_TRY_HIP(hipMemset(n->v, 0, sizeof(float) * MLP_NPARAM), "cm_mlp_set_params");
    n->step = 0;
    return CM_OK;
}

cm_status cm_mlp_infer(cm_mlp* n, const float* X, float* out, int batch, void* stream)
{
    cm_status st = check_net(n, "cm_mlp_infer");
    if (st != CM_OK) return st;
    if (!X || !out || batch < 1) { set_error("cm_mlp_infer: bad arguments"); return CM_ERR_ARG; }
    CM_TRY_HIP(hipSetDevice(n->device), "hipSetDevice");
    CM_TRY_HIP(ensure_capacity(n, batch), "cm_mlp_infer");
    CM_TRY_HIP(forward(n, X, batch, out, (hipStream_t)stream), "cm_mlp_infer");
    return CM_OK;
}

cm_status cm_mlp_grads(cm_mlp* n, const float* X, const float* T, int batch, float* grad_host, void* stream)
{
    cm_status st = check_net(n, "cm_mlp_grads");
    if (st != CM_OK) return st;
    if (!X || !T || !grad_host || batch < 1) { set_error("cm_mlp_grads: bad arguments"); return CM_ERR_ARG; }
    CM_TRY_HIP(hipSetDevice(n->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    CM_TRY_HIP(ensure_capacity(n, batch), "cm_mlp_grads");
    CM_TRY_HIP(forward(n, X, batch, n->O, s), "cm_mlp_grads forward");
    int nblk = 0;
    CM_TRY_HIP(backward(n, X, T, batch, &nblk, s), "cm_mlp_grads backward");
    CM_TRY_HIP(hipMemcpyAsync(grad_host, n->g, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost, s), "copy");
    CM_TRY_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    return CM_OK;
}

cm_status cm_mlp_train_step(cm_mlp* n, const float* X, const float* T, int batch, float* loss_host, void* stream)
{
    cm_status st = check_net(n, "cm_mlp_train_step");
    if (st != CM_OK) return st;
    if (!X || !T || batch < 1) { set_error("cm_mlp_train_step: bad arguments"); return CM_ERR_ARG; }
    CM_TRY_HIP(hipSetDevice(n->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    CM_TRY_HIP(ensure_capacity(n, batch), "cm_mlp_train_step");
    CM_TRY_HIP(forward(n, X, batch, n->O, s), "cm_mlp_train_step forward");
    int nblk = 0;
    CM_TRY_HIP(backward(n, X, T, batch, &nblk, s), "cm_mlp_train_step backward");
    n->step += 1;
    const float c1 = 1.0f - std::pow(n->desc.beta1, (float)n->step);
    const float c2 = 1.0f - std::pow(n->desc.beta2, (float)n->step);
    hipLaunchKernelGGL(k_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, MLP_NPARAM, n->p, n->g, n->m, n->v,
                       n->desc.lr, n->desc.beta1, n->desc.beta2, n->desc.eps, c1, c2);
    CM_TRY_HIP(hipGetLastError(), "k_adam");
    if (loss_host) {
        std::vector<float> part(nblk);
        CM_TRY_HIP(hipMemcpyAsync(part.data(), n->part, sizeof(float) * nblk, hipMemcpyDeviceToHost, s), "copy");
        CM_TRY_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
        double acc = 0.0;
        for (float v : part) acc += v;
        *loss_host = (float)(acc / batch);
    }
    return CM_OK;
}

// Weights of the fused closure: B fragments of every layer in lane order
// (see mlp_common.hpp), biases, and the input normalisation.
cm_status cm_model_set_mlp(cm_model* m, const float* params, const float* norm)
{
    if (!m || !params || !norm) { set_error("cm_model_set_mlp: null argument"); return CM_ERR_ARG; }
    if (m->desc.closure != CM_CLOSURE_MLP) {
        set_error("cm_model_set_mlp: the model's closure is not CM_CLOSURE_MLP");
        return CM_ERR_STATE;
    }
    for (int q = 0; q < 12; ++q)
        if (!(norm[12 + q] > 0.0f) || !(norm[36 + q] >= norm[24 + q])) {
            set_error("cm_model_set_mlp: need std > 0 and hi >= lo for every input");
            return CM_ERR_ARG;
        }
    CM_TRY_HIP(hipSetDevice(m->grid->device), "hipSetDevice");
    // A-operand tiles of W [out][in] for the transposed forward (zero
    // outside the matrix).  Layer 1, 16x16x16 tile ht: lane l, element q holds
    // W[16 ht + l % 16][4 (l / 16) + q].  Layers 2-4, 16x16x32 tile (ht, chunk
    // c): lane l, slot s holds W[16 ht + l % 16][32 c + k32_unit(l / 16, s)].
    std::vector<uint16_t> frag((size_t)FRAG_TOTAL * 64 * 4, 0);
    struct L { int off, nin, nout, ht, base; } layers[4] = {
        {OFF_W1, MLP_NI, MLP_NH, 4, 0}, {OFF_W2, MLP_NH, MLP_NH, 4, FRAG_L1},
        {OFF_W3, MLP_NH, MLP_NH, 4, FRAG_L1 + FRAG_L2}, {OFF_W4, MLP_NH, MLP_NO, 1, FRAG_L1 + FRAG_L2 + FRAG_L3}};
    auto wbf = [&](const L& l, int j, int k) {
        return f2bf((j < l.nout && k < l.nin) ? params[l.off + j * l.nin + k] : 0.0f);
    };
    for (int ht = 0; ht < 4; ++ht)
        for (int lane = 0; lane < 64; ++lane)
            for (int q = 0; q < 4; ++q)
                frag[((size_t)ht * 64 + lane) * 4 + q] = wbf(layers[0], ht * 16 + (lane & 15), 4 * (lane >> 4) + q);
    for (int li = 1; li < 4; ++li) {
        const L& l = layers[li];
        for (int ht = 0; ht < l.ht; ++ht)
            for (int c = 0; c < 2; ++c)
                for (int lane = 0; lane < 64; ++lane)
                    for (int s = 0; s < 8; ++s) {
                        const size_t unit = (size_t)l.base + 2 * (2 * ht + c);
                        frag[unit * 64 * 4 + (size_t)lane * 8 + s] =
                            wbf(l, ht * 16 + (lane & 15), 32 * c + k32_unit(lane >> 4, s));
                    }
    }
    std::vector<float> bias(3 * MLP_NH + 16, 0.0f);
    for (int q = 0; q < MLP_NH; ++q) {
        bias[q] = params[OFF_B1 + q];
        bias[MLP_NH + q] = params[OFF_B2 + q];
        bias[2 * MLP_NH + q] = params[OFF_B3 + q];
    }
    bias[3 * MLP_NH + 0] = params[OFF_B4 + 0];
    bias[3 * MLP_NH + 1] = params[OFF_B4 + 1];
    // device copy: mean[12], std[12], centre of the standardised training
    // range[12], allowed distance from the centre[12] = 1.1 x half-width plus
    // 2^-20 (1 + |mean/std|) (the float rounding of the normalisation, so an
    // input that was constant in training passes at its training value),
    // 1 / std[12]
    std::vector<double> nrm(60);
    for (int q = 0; q < 12; ++q) {
        const double mean = norm[q], sd = norm[12 + q], lo = norm[24 + q], hi = norm[36 + q];
        nrm[q] = mean;
        nrm[12 + q] = sd;
        nrm[24 + q] = 0.5 * (lo + hi);
        nrm[36 + q] = 1.1 * (0.5 * (hi - lo)) + std::ldexp(1.0 + std::fabs(mean / sd), -20);
        nrm[48 + q] = 1.0 / sd;
    }
    if (!m->d_mlp_w) {
        const size_t bytes = frag.size() * sizeof(uint16_t) + bias.size() * sizeof(float);
        CM_TRY_HIP(hipMalloc(&m->d_mlp_w, bytes), "cm_model_set_mlp");
        CM_TRY_HIP(hipMalloc(&m->d_mlp_norm, sizeof(double) * 60), "cm_model_set_mlp");
    }
    uint16_t* dfrag = (uint16_t*)m->d_mlp_w;
    float* dbias = (float*)(dfrag + frag.size());
    CM_TRY_HIP(hipMemcpy(dfrag, frag.data(), frag.size() * sizeof(uint16_t), hipMemcpyHostToDevice), "copy");
    CM_TRY_HIP(hipMemcpy(dbias, bias.data(), bias.size() * sizeof(float), hipMemcpyHostToDevice), "copy");
    CM_TRY_HIP(hipMemcpy(m->d_mlp_norm, nrm.data(), sizeof(double) * 60, hipMemcpyHostToDevice), "copy");
    m->kp.mlp_frag = dfrag;
    m->kp.mlp_bias = dbias;
    m->kp.mlp_norm = m->d_mlp_norm;
    m->mlp_ready = 1;
    return CM_OK;
}

cm_status cm_model_mlp_fallbacks(cm_model* m, int64_t* count, void* stream)
{
    if (!m || !count) { set_error("cm_model_mlp_fallbacks: null argument"); return CM_ERR_ARG; }
    CM_TRY_HIP(hipSetDevice(m->grid->device), "hipSetDevice");
    unsigned long long c = 0;
    CM_TRY_HIP(hipMemcpyAsync(&c, m->d_fallbacks, sizeof(c), hipMemcpyDeviceToHost, (hipStream_t)stream), "copy");
    CM_TRY_HIP(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
    CM_TRY_HIP(hipMemsetAsync(m->d_fallbacks, 0, sizeof(c), (hipStream_t)stream), "reset");
    *count = (int64_t)c;
    return CM_OK;
}

}  // extern "C"
