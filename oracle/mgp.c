/*
 * Oracle integrands of the MGP kernel correction (TEST INFRASTRUCTURE ONLY;
 * nothing on the product path links or calls this file).
 *
 * Section "New-generation nonlocal KEDFs", eq. "MGP":
 *   I(eta) = int_0^1 dt t^y d/dt G_NL(eta(q, t)),  eta(q, t) = eta t^(-1/3)
 * (the reading of eta(q, t) is stated in oracle/mgp.py).  With t = s^3,
 *   I(eta) = -eta int_0^1 s^(3y-2) G'(eta / s) ds,
 * and, for eta < 1, the part s < eta (where the argument exceeds 1) is
 * rescaled by s = eta r:
 *   -eta int_0^eta s^(3y-2) G'(eta/s) ds = -eta^(3y) int_0^1 r^(3y-2) G'(1/r) dr.
 * The functions below are those integrands in the form scipy's quad takes
 * from a LowLevelCallable, double f(int n, double *x): x[0] the variable,
 * x[1] = eta, x[2] = y.
 *
 * G(e) = 1/F(e) - 3 e^2 - 1 with F(e) = 1/2 + (1 - e^2)/(4 e) ln|(1+e)/(1-e)|
 * (the printed G_NL).  Expanding atanh, F = 1 - sum_{k>=1} c_k e^(2k) below
 * e = 1 and F = sum_{k>=1} c_k e^(-2k) above, c_k = 1/((2k-1)(2k+1)); the
 * series are used where they converge fast (e < 1/2, e > 3/2), the closed
 * form in between.  G' = -F'/F^2 - 6 e; above 3/2 the cancellation-free form
 * G = -1 - S(u)/P(u), u = 1/e^2, P = sum c_k u^(k-1), S = sum 3 c_k u^(k-2)
 * (k >= 2), is differentiated instead.
 */
#include <math.h>

static double ck(int k) { return 1.0 / ((2.0 * k - 1.0) * (2.0 * k + 1.0)); }

/* G'(e) for e > 0, e != 1 */
double oracle_dgnl(double e)
{
    if (e < 0.5) {
        double F = 1.0, dF = 0.0, p = e;     /* p = e^(2k-1) */
        for (int k = 1; k <= 40; ++k) {
            const double c = ck(k);
            dF -= 2.0 * k * c * p;
            p *= e;
            F -= c * p;
            p *= e;
        }
        return -dF / (F * F) - 6.0 * e;
    }
    if (e <= 1.5) {
        const double L = log(fabs((1.0 + e) / (1.0 - e)));
        const double F = 0.5 + (1.0 - e * e) / (4.0 * e) * L;
        const double dF = -(1.0 + e * e) * L / (4.0 * e * e) + 1.0 / (2.0 * e);
        return -dF / (F * F) - 6.0 * e;
    }
    const double u = 1.0 / (e * e);
    double P = 0.0, dP = 0.0, S = 0.0, dS = 0.0;
    for (int k = 60; k >= 1; --k) {          /* Horner for P and dP/du */
        dP = dP * u + P;
        P = P * u + ck(k);
    }
    for (int k = 60; k >= 2; --k) {
        dS = dS * u + S;
        S = S * u + 3.0 * ck(k);
    }
    const double dGdu = -(dS * P - S * dP) / (P * P);
    return dGdu * (-2.0 / (e * e * e));
}

/* -eta s^(3y-2) G'(eta/s) */
double oracle_mgp_upper(int n, double *x)
{
    (void)n;
    const double s = x[0], eta = x[1], y = x[2];
    if (s <= 0.0) return 0.0;
    const double a = eta / s;
    if (a == 1.0) return 0.0;   /* integrable logarithmic singularity */
    return -eta * pow(s, 3.0 * y - 2.0) * oracle_dgnl(a);
}

/* -r^(3y-2) G'(1/r) (the s < eta part, to be multiplied by eta^(3y)) */
double oracle_mgp_lower(int n, double *x)
{
    (void)n;
    const double r = x[0], y = x[2];
    if (r <= 0.0 || r >= 1.0) return 0.0;
    return -pow(r, 3.0 * y - 2.0) * oracle_dgnl(1.0 / r);
}
