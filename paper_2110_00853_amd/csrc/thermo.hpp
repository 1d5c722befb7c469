// Device thermodynamics (Sects. 2.4-2.7, Table 1), always FP64: recovery of
// velocity, temperature, pressure, sound speed and total enthalpy from the
// conserved state; the saturation adjustment (Newton iteration with the
// analytic derivative of the equilibrium internal energy), liquid only or
// with the condensate split between liquid and ice by temperature; the
// virtual potential temperature.  Shared by the DG passes and the
// diagnostics reduction.
#pragma once

#include "cm_impl.hpp"
#include "fp64_math.hpp"

namespace cm {

// qc is the total condensate q_l + q_i (all liquid without the ice phase)
struct Th {
    double rho, u, v, w, e, qt, T, p, c, h, qv, qc, Rm;
};

__device__ __forceinline__ double pvsat(double T)
{
    // Clausius-Clapeyron integrated with constant heat capacities:
    // p* = p_tr (T/T0)^((c_pv-c_pl)/R_v) exp((L_v0-(c_pv-c_pl)T0)/R_v (1/T0 - 1/T))
    constexpr double dc = Phys::cpv - Phys::cpl;
    return Phys::ptr * exp_fin(dc / Phys::Rv * ln_pos(T * (1.0 / Phys::T0)) +
                               (Phys::Lv0 - dc * Phys::T0) / Phys::Rv * (1.0 / Phys::T0 - frcp(T)));
}

// over ice: latent heat of sublimation L_v0 + L_f0 at T0, c_vi for the ice
__device__ __forceinline__ double pvsat_ice(double T)
{
    constexpr double dc = Phys::cpv - Phys::cvi;
    return Phys::ptr * exp_fin(dc / Phys::Rv * ln_pos(T * (1.0 / Phys::T0)) +
                               (Phys::Lv0 + Phys::Lf0 - dc * Phys::T0) / Phys::Rv * (1.0 / Phys::T0 - frcp(T)));
}

// liquid fraction of the condensate: 1 at and above freezing, 0 at and
// below homogeneous nucleation, linear in between (the paper says only that
// the split follows temperature)
__device__ __forceinline__ double liquid_fraction(double T)
{
    constexpr double inv = 1.0 / (Phys::T_freeze - Phys::T_icenuc);
    return T >= Phys::T_freeze ? 1.0 : (T <= Phys::T_icenuc ? 0.0 : (T - Phys::T_icenuc) * inv);
}

// saturation vapour pressure over the mix (liquid fraction lam) and its
// derivative d p*/dT
__device__ __forceinline__ void pvsat_mix(double T, double& pv, double& dpv)
{
    const double iT = frcp(T), dT = T - Phys::T0;
    const double pl = pvsat(T), pi = pvsat_ice(T);
    const double lam = liquid_fraction(T);
    const double dlam = (T > Phys::T_icenuc && T < Phys::T_freeze) ? 1.0 / (Phys::T_freeze - Phys::T_icenuc) : 0.0;
    const double Lv = Phys::Lv0 + (Phys::cpv - Phys::cpl) * dT;
    const double Ls = Phys::Lv0 + Phys::Lf0 + (Phys::cpv - Phys::cvi) * dT;
    const double k = (1.0 / Phys::Rv) * iT * iT;
    pv = lam * pl + (1.0 - lam) * pi;
    dpv = lam * pl * Lv * k + (1.0 - lam) * pi * Ls * k + dlam * (pl - pi);
}

// equilibrium temperature with the ice phase: Newton on I*(T) - I with the
// analytic derivative, kept inside a bracket (the liquid fraction has kinks
// at the ramp's ends, where a Newton step may overshoot: then bisection);
// starts from Tg when that lies above T_u.  qc: q_t - q_v* at the result.
__device__ __forceinline__ double sat_adjust_ice(double rho, double qt, double I, double Tu, double Tg, double& qc)
{
    const double irv = frcp(rho * Phys::Rv);
    double lo = Tu, hi = Tu + (Phys::Lv0 + Phys::Lf0) * qt * (1.0 / Phys::cvd);
    double Tn = Tg > Tu && Tg < hi ? Tg : Tu;
    for (int it = 0; it < 40; ++it) {
        double pv, dpv;
        pvsat_mix(Tn, pv, dpv);
        const double iT = frcp(Tn);
        const double qv = pv * irv * iT;
        const double qcn = qt - qv;
        const double lam = liquid_fraction(Tn);
        const double dT = Tn - Phys::T0;
        const double f = (1.0 - qt) * Phys::cvd * dT + qv * (Phys::cvv * dT + Phys::Iv0) +
                         qcn * (lam * Phys::cvl * dT + (1.0 - lam) * (Phys::cvi * dT - Phys::Lf0)) - I;
        if (f < 0.0) lo = Tn; else hi = Tn;
        const double dqv = qv * (dpv * frcp(pv) - iT);
        const double dlam = (Tn > Phys::T_icenuc && Tn < Phys::T_freeze) ? 1.0 / (Phys::T_freeze - Phys::T_icenuc) : 0.0;
        const double cvm = (1.0 - qt) * Phys::cvd + qv * Phys::cvv + qcn * (lam * Phys::cvl + (1.0 - lam) * Phys::cvi);
        const double fp = cvm + dqv * (Phys::cvv * dT + Phys::Iv0 - lam * Phys::cvl * dT - (1.0 - lam) * (Phys::cvi * dT - Phys::Lf0)) +
                          qcn * dlam * ((Phys::cvl - Phys::cvi) * dT + Phys::Lf0);
        // the bracket's ends count as inside: at an exact root (f = 0) the
        // iterate is itself an end, and the zero step must stand
        double Tnew = Tn - f * frcp(fp);
        if (!(Tnew >= lo && Tnew <= hi)) Tnew = 0.5 * (lo + hi);
        const double step = Tnew - Tn;
        Tn = Tnew;
        if (fabs(step) <= 1e-13 * Tn) break;
    }
    double pv, dpv;
    pvsat_mix(Tn, pv, dpv);
    double qv = pv * irv * frcp(Tn);
    qv = qv < qt ? qv : qt;
    qc = qt - qv;
    return Tn;
}

// Saturation adjustment: T from (rho, q_t, I) by Newton iteration with the
// analytic derivative dI*/dT; unsaturated air returns T_u directly.  qc is
// the condensate at the result.
__device__ __forceinline__ void saturation_adjust(double rho, double qt, double I, bool ice, double& T, double& qc)
{
    const double Tu = Phys::T0 + (I - qt * Phys::Iv0) * frcp((1.0 - qt) * Phys::cvd + qt * Phys::cvv);
    const double irv = frcp(rho * Phys::Rv);
    if (ice) {
        double pv, dpv;
        pvsat_mix(Tu, pv, dpv);
        if (qt <= pv * irv * frcp(Tu)) { T = Tu; qc = 0.0; return; }
        T = sat_adjust_ice(rho, qt, I, Tu, Tu, qc);
        return;
    }
    const double qvs_u = pvsat(Tu) * irv * frcp(Tu);
    if (qt <= qvs_u) { T = Tu; qc = 0.0; return; }
    double Tn = Tu;
    for (int it = 0; it < 20; ++it) {
        const double iT = frcp(Tn);
        const double qv = pvsat(Tn) * irv * iT;
        const double dT = Tn - Phys::T0;
        const double f = (1.0 - qt) * Phys::cvd * dT + qv * (Phys::cvv * dT + Phys::Iv0) + (qt - qv) * Phys::cvl * dT - I;
        const double Lv = Phys::Lv0 + (Phys::cpv - Phys::cpl) * dT;
        const double dqv = qv * (Lv * (1.0 / Phys::Rv) * iT * iT - iT);
        const double cvm = (1.0 - qt) * Phys::cvd + qv * Phys::cvv + (qt - qv) * Phys::cvl;
        const double fp = cvm + dqv * (Phys::Iv0 + (Phys::cvv - Phys::cvl) * dT);
        const double step = f * frcp(fp);
        Tn -= step;
        if (fabs(step) <= 1e-13 * Tn) break;
    }
    double qv = pvsat(Tn) * irv * frcp(Tn);
    qv = qv < qt ? qv : qt;
    T = Tn;
    qc = qt - qv;
}

// condensate of a moist state at its adjusted temperature T: the
// adjustment's own q_v = min(q_t, q_v*(T)), for the unsaturated branch as well
__device__ __forceinline__ double moist_qc(double rho, double rq, double T, bool ice)
{
    const double qt = rq * frcp(rho);
    const double irv = frcp(rho * Phys::Rv);
    double pv;
    if (ice) {
        double dpv;
        pvsat_mix(T, pv, dpv);
    } else {
        pv = pvsat(T);
    }
    double qv = pv * irv * frcp(T);
    qv = qv < qt ? qv : qt;
    return qt - qv;
}

// gas constant, pressure, sound speed and enthalpy of a moist state from
// its temperature and condensate (liquid and ice split by the liquid
// fraction with the ice phase, all liquid without)
__device__ __forceinline__ void moist_eos(double rho, double ir, bool ice, Th& o)
{
    o.qv = o.qt - o.qc;
    o.Rm = Phys::Rd * (1.0 - o.qt) + Phys::Rv * o.qv;
    const double lam = ice ? liquid_fraction(o.T) : 1.0;
    const double cvm = (1.0 - o.qt) * Phys::cvd + o.qv * Phys::cvv + o.qc * (lam * Phys::cvl + (1.0 - lam) * Phys::cvi);
    o.p = rho * o.Rm * o.T;
    o.c = fsqrt((cvm + o.Rm) * frcp(cvm) * o.Rm * o.T);
    o.h = o.e + o.p * ir;
}

// the moist recovery when T and the condensate are already known (the
// saturation adjustment of the same state earlier in the stage or step):
// the same values thermo() gives, without the Newton iteration or q_v*
__device__ __forceinline__ void thermo_moist_T(double rho, double mx, double my, double mz, double re, double rq,
                                               double T, double qc, bool ice, Th& o)
{
    const double ir = frcp(rho);
    o.rho = rho;
    o.u = mx * ir; o.v = my * ir; o.w = mz * ir;
    o.e = re * ir;
    o.qt = rq * ir;
    o.T = T;
    o.qc = qc;
    moist_eos(rho, ir, ice, o);
}

// temperature of a moist state by the saturation adjustment, Newton
// started from Tg when that is above T_u (a nearby solution: the previous
// stage's temperature of the same node); unsaturated air returns T_u.  qc
// is the condensate at the returned temperature, as moist_qc gives it
// (zero for unsaturated air without a second q_v* evaluation: there
// moist_qc's minimum picks q_t)
__device__ __forceinline__ double moist_T_guess(double rho, double mx, double my, double mz, double re, double rq,
                                                double z, double g, double Tg, bool ice, double& qc)
{
    const double ir = frcp(rho);
    const double u = mx * ir, v = my * ir, w = mz * ir;
    const double I = re * ir - 0.5 * (u * u + v * v + w * w) - g * z;
    const double qt = rq * ir;
    const double Tu = Phys::T0 + (I - qt * Phys::Iv0) * frcp((1.0 - qt) * Phys::cvd + qt * Phys::cvv);
    const double irv = frcp(rho * Phys::Rv);
    qc = 0.0;
    if (ice) {
        double pv, dpv;
        pvsat_mix(Tu, pv, dpv);
        if (qt <= pv * irv * frcp(Tu)) return Tu;
        return sat_adjust_ice(rho, qt, I, Tu, Tg, qc);
    }
    const double qvs_u = pvsat(Tu) * irv * frcp(Tu);
    if (qt <= qvs_u) return Tu;
    double Tn = Tg > Tu ? Tg : Tu;
    for (int it = 0; it < 20; ++it) {
        const double iT = frcp(Tn);
        const double qv = pvsat(Tn) * irv * iT;
        const double dT = Tn - Phys::T0;
        const double f = (1.0 - qt) * Phys::cvd * dT + qv * (Phys::cvv * dT + Phys::Iv0) + (qt - qv) * Phys::cvl * dT - I;
        const double Lv = Phys::Lv0 + (Phys::cpv - Phys::cpl) * dT;
        const double dqv = qv * (Lv * (1.0 / Phys::Rv) * iT * iT - iT);
        const double cvm = (1.0 - qt) * Phys::cvd + qv * Phys::cvv + (qt - qv) * Phys::cvl;
        const double fp = cvm + dqv * (Phys::Iv0 + (Phys::cvv - Phys::cvl) * dT);
        const double step = f * frcp(fp);
        Tn -= step;
        if (fabs(step) <= 1e-13 * Tn) break;
    }
    qc = moist_qc(rho, rq, Tn, false);
    return Tn;
}

template <bool MOIST>
__device__ __forceinline__ void thermo(double rho, double mx, double my, double mz, double re, double rq, double z,
                                       double g, bool ice, Th& o)
{
    const double ir = frcp(rho);
    o.rho = rho;
    o.u = mx * ir; o.v = my * ir; o.w = mz * ir;
    o.e = re * ir;
    const double I = o.e - 0.5 * (o.u * o.u + o.v * o.v + o.w * o.w) - g * z;
    if (MOIST) {
        o.qt = rq * ir;
        saturation_adjust(rho, o.qt, I, ice, o.T, o.qc);
        moist_eos(rho, ir, ice, o);
    } else {
        o.qt = 0.0; o.qc = 0.0; o.qv = 0.0;
        o.T = Phys::T0 + I * (1.0 / Phys::cvd);
        o.Rm = Phys::Rd;
        o.p = rho * Phys::Rd * o.T;
        o.c = fsqrt(Phys::cpd / Phys::cvd * Phys::Rd * o.T);
        o.h = o.e + o.p * ir;
    }
}

// virtual potential temperature theta_v = T (p0/p)^(R_d/c_pd) R_m/R_d, in the
// storage precision: FP64, or with FP32-bulk storage in FP32 from the FP64
// T and p (it only enters the Richardson number; pressure and temperature
// themselves stay FP64)
template <typename R> __device__ __forceinline__ R theta_v(const Th& o);
template <> __device__ __forceinline__ double theta_v<double>(const Th& o)
{
    return o.T * exp_fin(Phys::kappa * ln_pos(Phys::p0 * frcp(o.p))) * (o.Rm * (1.0 / Phys::Rd));
}
template <> __device__ __forceinline__ float theta_v<float>(const Th& o)
{
    const float x = (float)(Phys::p0 / o.p);
    return (float)o.T * __expf((float)Phys::kappa * __logf(x)) * (float)(o.Rm * (1.0 / Phys::Rd));
}

}  // namespace cm
