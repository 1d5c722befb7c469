/*
 * Learned SGS closure: reference forward pass (TEST INFRASTRUCTURE ONLY).
 * Placeholder until the network oracle is written: every node falls back to
 * the Smagorinsky-Lilly viscosity.
 */
int cmref_mlp_closure(const double* params, const double* lo, const double* hi, int use_fallback,
                      const double gu[3][3], double N2, double Delta, double nu_sl,
                      double* nu, double* Prt)
{
    (void)params; (void)lo; (void)hi; (void)use_fallback; (void)gu; (void)N2; (void)Delta;
    *nu = nu_sl; *Prt = 1.0 / 3.0;
    return 1;
}
