// Internal declarations of the gfx950 DG LES library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cm.h"

namespace cm {

constexpr int NQ = 5;            // GLL points per direction (N = 4)
constexpr int NP = NQ * NQ * NQ; // nodes per element
constexpr int BLOCK = 128;       // two wave64 per element

// ---- thermodynamic constants: Table 1, and the readings g, p0,
//      c_pd = c_vd + R_d, triple-point pressure of water --------------------
struct Phys {
    static constexpr double Rd = 287.0, Rv = 462.0;
    static constexpr double cvd = 717.5, cvv = 1397.5, cvl = 4181.0;
    static constexpr double T0 = 273.16;
    static constexpr double Lv0 = 2.5008e6;
    static constexpr double p0 = 1.0e5;
    static constexpr double ptr = 611.657;
    static constexpr double cpd = cvd + Rd;
    static constexpr double cpv = cvv + Rv;
    static constexpr double cpl = cvl;
    static constexpr double Iv0 = Lv0 - Rv * T0;
    static constexpr double kappa = Rd / cpd;
    // ice (Table 1: c_vi, L_f0 = I_i0) and the liquid-fraction ramp
    static constexpr double cvi = 2100.0, Lf0 = 0.3336e6;
    static constexpr double T_freeze = 273.15, T_icenuc = 233.0;
};

// Everything the kernels need, passed by value.
// nodes per element run in the model-owned per-node arrays (stored
// diffusive flux, carried temperatures): 125 used, padded so that every run
// starts on a 128-byte line and the two waves of a block write whole lines
// (nodes 0-63, 64-127); 144 (FP64) and 160 (FP32) keep the run stride off a
// power of two
#ifndef CM_F2RUN64
#define CM_F2RUN64 144
#endif
template <typename R> constexpr int run_nodes() { return sizeof(R) == 8 ? CM_F2RUN64 : 160; }

// slots per element in the state buffers (Y, dQ, dY/dt): the element's 125
// nodes, then padding, so that every element run starts on a 128-byte line
// in both precisions (1280 / 640 bytes) and a block's stores cover whole
// lines (the lanes beyond the element write zeros); a stride off a power of
// two
#ifndef CM_SRUN
#define CM_SRUN 160
#endif
constexpr int SRUN = CM_SRUN;

struct KParams {
    int ne0, ne1, ne2;
    int per0, per1, per2;
    int n_elem;
    const int* order;           // per-XCD element traversal table [n_elem]
    int64_t nn;                 // nodes
    int64_t nnS;                // stride of one state variable: n_elem x SRUN
    double lo0, lo1, lo2;
    double h0, h1, h2;          // element extents (Cartesian metrics)
    double r2h0, r2h1, r2h2;    // 2 / h_d
    double lift0, lift1, lift2; // 2 / (h_d w_N): J^s / (J w_N) on flat meshes
    double zgll[NQ];            // (1 + xi_k)/2
    int warped;
    const void* metrics;        // warped: [10][nn] = J a^d_c (9), 1/J  (storage type)
    const double* zn;           // warped: node heights [nn]
    // reference state: either per level (flat, horizontally uniform) or per node
    const double* pr;           // reference pressure
    const double* rhor;         // reference density
    int ref_per_node;
    int has_ref;
    // FP32-bulk storage holds each state as its deviation from the
    // background: the background [nvar][nref] (float, indexed like pr), null
    // for FP64 models, whose states hold full values
    const float* bg32;
    int64_t nref;
    // physics
    double g;
    int closure;
    double nu, Cs, Prt, invPrt, Delta;
    int richardson;
    double f_cor, u_g, v_g;
    int sponge;
    double sp_zs, sp_ztop, sp_alpha, sp_gamma, sp_u0, sp_u1, sp_u2, sp_inv;
    int sfc_flux;
    double theta_flux, qt_flux;
    int subsidence;
    double sub_w0, sub_ztop, sub_inv;
    int ice;  // moist: condensate split between liquid and ice by temperature
    int nf;                     // words per node of the stored diffusive flux
    int64_t nnf;                // stride of one F2 word: n_elem x F2_RUN (padded element runs)
    // learned closure
    const uint16_t* mlp_frag;   // bf16 B fragments of the four layers
    const float* mlp_bias;      // biases: 64, 64, 64, 2 (padded to 16)
    const double* mlp_norm;     // mean[12], std[12], range centre[12], allowed distance from it[12], 1/std[12]
    int mlp_fallback_on;
    unsigned long long* mlp_fallbacks;
    double* feat_out;           // when set, the gradient pass also writes the closure inputs [nn][16]
    // moist viscous models: node temperature of the stage's input state
    // (written by the gradient pass, or by the previous stage's tendency
    // pass when T_given) and of its output state (written by the tendency
    // pass when Tnext is set) [nn]
    // Each buffer holds T at [0, nnT) and q_l at [nnT, 2 nnT), in padded runs.
    double* Tn;
    double* Tnext;
    int T_given;
    int64_t nnT;
    // per-variable / per-word array bases of the current launch (filled on
    // the host): state input, output, dQ, stored diffusive flux
    const void* Ys[6];
    void* outs[6];
    void* dQs[6];
    void* F2s[14];
};

}  // namespace cm

struct cm_grid {
    int device = 0;
    cm_grid_desc desc{};
    int64_t n_elem = 0, n_nodes = 0;
    double h[3] = {0, 0, 0};
    double xi[cm::NQ], w[cm::NQ], D[cm::NQ * cm::NQ];
    std::vector<double> xyz;     // host [3][nn]
    std::vector<double> Ja, J;   // host [9][nn], [nn]
    double* d_metrics64 = nullptr;  // warped only: [10][nn]
    float* d_metrics32 = nullptr;
    double* d_z = nullptr;          // warped only: node heights
    int* d_order = nullptr;         // element traversal table [n_elem]
    int n_cu = 0;                   // compute units of the device
    double dmin = 0.0;
};

struct cm_model {
    const cm_grid* grid = nullptr;
    int device = 0;              // the grid's device, kept so that destroy never reads the grid
    cm_model_desc desc{};
    int nf = 0;
    void* d_F2 = nullptr;        // [nf][nn] storage type
    double* d_T[2] = {nullptr, nullptr};  // moist viscous models: node T and q_l, ping-pong
    int tsel = 0;                // which d_T holds the current stage input's T
    double* d_pr = nullptr;
    double* d_rhor = nullptr;
    double* d_Yref = nullptr;    // the background itself [nvar][nref] (per level or per node; zeros without one)
    float* d_bg32 = nullptr;     // FP32-bulk models: the same background in float (its values are floats)
    double* d_bg64 = nullptr;    // FP32-bulk models with a background: the background as given (state import/export)
    int64_t nref = 0;            // entries per variable of the background tables
    int ref_per_node = 0;
    int has_ref = 0;
    double Delta = 0.0;
    // diagnostics scratch
    double* d_partials = nullptr;
    int n_partials = 0;
    // learned closure
    void* d_mlp_w = nullptr;
    double* d_mlp_norm = nullptr;
    unsigned long long* d_fallbacks = nullptr;
    int mlp_ready = 0;
    // 1-D IMEX: the line factor shared by every vertical line (models with a
    // per-level background on flat meshes) and the tau it was formed for
    double* d_hevi_fac = nullptr;
    double hevi_fac_tau = -1.0;
    cm::KParams kp{};
    // optional per-launch event timing
    struct ProfRec {
        hipEvent_t a, b;
        int kind;
    };
    std::vector<ProfRec> prof;
    size_t prof_used = 0;
    int profiling = 0;
};

namespace cm {
void set_error(const std::string& msg);
cm_status hip_fail(hipError_t e, const char* where);

// kernel launchers (dg_kernels.hip)
hipError_t launch_reference(const cm_model* m, const double* Yref_dev, hipStream_t s);
hipError_t launch_rhs(cm_model* m, const void* Y, void* out, void* dQ, int mode, double A, double B,
                      double dt, hipStream_t s);
hipError_t launch_grad_only(cm_model* m, const void* Y, hipStream_t s);
hipError_t upload_constants(const cm_grid* g);
// event brackets around one launch when profiling is on
cm_model::ProfRec* prof_begin(cm_model* m, int kind, hipStream_t s);
void prof_end(cm_model::ProfRec* r, hipStream_t s);
// reductions (reduce.hip)
hipError_t launch_diagnostics(const cm_model* m, const void* Y, double dt, cm_diag* out, hipStream_t s);
// 1-D IMEX (hevi.hip): the linear vertical operator (Lout = L(Y - Y_ref),
// Eout -= Lout when given), the line solves, and out = base + sum c_q X_q
hipError_t launch_hevi_operator(const cm_model* m, const void* Y, void* Lout, void* Eout, hipStream_t s);
hipError_t launch_hevi_solve(cm_model* m, double tau, const void* B, void* Yout, double* scratch, hipStream_t s);
size_t hevi_factor_doubles(int nz);
hipError_t launch_combine(const cm_model* m, const void* base, void* out, int n, const double* c, const void* const* X,
                          hipStream_t s);
int64_t hevi_lines(const cm_model* m);
// exponential modal filter (filter.hip): F1 the 1-D filter matrix [5][5]
hipError_t launch_exp_filter(const cm_model* m, void* Y, int mask, const double* F1, hipStream_t s);
hipError_t launch_state_convert(const cm_model* m, const void* src, void* dst, bool to_storage, hipStream_t s);
// the same reduction over the library's static per-device workspace (no
// allocation); its partial-record count equals a model's, so both give
// bit-identical results
constexpr int DIAG_SCRATCH_RECORDS = 2048;
hipError_t launch_diagnostics_static(const cm_model* m, const void* Y, double dt, cm_diag* out, hipStream_t s);
}  // namespace cm
