// vfp_impedance.hpp -- impedance samples computed on the device (included by
// vfp.hip after vfp_kernels.hpp).
//
// Z_k at kappa_k = k * dkappa, k = 0 .. nk-1, for the models the wake takes
// (Sec. II.B): free space, Z = F kappa^{1/3} (cos 30deg + i sin 30deg) with
// F = Gamma(2/3) / 3^{1/3}, and parallel plates (the normalised
// shielded-CSR impedance with P = Pi^{2/3}):
//   Z = 4 pi^2 2^{1/3} P kappa^{-1/3} sum_{p>=0} T(u_p),
//   u_p = A (2p+1)^2,  A = pi^2 2^{-2/3} P^2 kappa^{-4/3},
//   T(u) = Ai'(u) Ci'(u) + u Ai(u) Ci(u),  Ci = Ai - i Bi.
// Terms with u_p <= kUAsym are summed explicitly; beyond, T -> -i (3/(16 pi))
// u^{-5/2} and the remaining sum is (2p+1)^{-5} summed in closed form,
// 2^{-5} zeta(5, p* + 1/2) (Hurwitz zeta).  One thread per k, FP64.
//
// Airy functions for u > 0 (DLMF 9.7, 9.2):
//   u > kUAiry: the asymptotic expansions of Ai, Ai', Bi, Bi' in
//     zeta = (2/3) u^{3/2}; the products entering T need no exponentials
//     except the e^{-2 zeta} of Re T;
//   u <= kUAiry: Taylor stepping of y'' = x y (coefficients
//     c_{m+2} = (x0 c_m + c_{m-1}) / ((m+2)(m+1))): Ai and Ai' backward from
//     u = kUAiry (where the expansion is exact to rounding), the direction in
//     which Ai grows; Bi and Bi' forward from 0, the direction in which Bi
//     grows.
#pragma once

namespace vfp {

constexpr double kUAsym = 100.0;    // explicit terms up to this Airy argument
constexpr double kUAiry = 10.0;     // asymptotic Airy expansions above this argument
constexpr int kAiryTerms = 40;      // Taylor terms per step
constexpr double kAiryStep = 0.5;   // Taylor step length

// y(x0 + h), y'(x0 + h) for y'' = x y from y(x0), y'(x0)
__device__ inline void airy_taylor_step(double x0, double h, double &y, double &yp)
{
    double cm1 = 0.0, c0 = y, c1 = yp;          // c_{m-1}, c_m, c_{m+1} for m = 0
    double hp = 1.0;                             // h^m
    double sy = 0.0, syp = 0.0;
    for (int m = 0; m < kAiryTerms; ++m) {
        sy += c0 * hp;                           // c_m h^m
        syp += (m + 1) * c1 * hp;                // (m+1) c_{m+1} h^m
        const double c2 = (x0 * c0 + cm1) / ((m + 2.0) * (m + 1.0));
        cm1 = c0;
        c0 = c1;
        c1 = c2;
        hp *= h;
    }
    y = sy;
    yp = syp;
}

// asymptotic sums S_A, S_A', S_B, S_B' at zeta (DLMF 9.7.5-9.7.8)
__device__ inline void airy_asym_sums(double zeta, double &sa, double &sap, double &sb, double &sbp)
{
    double uk = 1.0, zk = 1.0;
    sa = sb = sap = sbp = 1.0;
    double prev = 1e300;
    for (int k = 1; k < 60; ++k) {
        uk *= (6.0 * k - 5.0) * (6.0 * k - 3.0) * (6.0 * k - 1.0) / ((2.0 * k - 1.0) * 216.0 * k);
        const double vk = -uk * (6.0 * k + 1.0) / (6.0 * k - 1.0);
        zk /= zeta;
        const double tu = uk * zk, tv = vk * zk;
        if (fabs(tu) > prev) break;              // the expansion started to diverge
        prev = fabs(tu);
        const double sg = (k & 1) ? -1.0 : 1.0;
        sa += sg * tu;
        sb += tu;
        sap += sg * tv;
        sbp += tv;
        if (fabs(tu) < 1e-18 && fabs(tv) < 1e-18) break;
    }
}

// Ai, Ai' at u in (0, kUAiry] by backward stepping from kUAiry
__device__ inline void airy_ai_small(double u, double &ai, double &aip)
{
    const double x1 = kUAiry, z1 = (2.0 / 3.0) * x1 * sqrt(x1), q1 = sqrt(sqrt(x1));
    double sa, sap, sb, sbp;
    airy_asym_sums(z1, sa, sap, sb, sbp);
    const double e = exp(-z1) / (2.0 * sqrt(M_PI));
    double y = e / q1 * sa, yp = -e * q1 * sap;
    const int steps = (int)ceil((x1 - u) / kAiryStep);
    const double h = (u - x1) / steps;
    double x = x1;
    for (int s = 0; s < steps; ++s, x += h) airy_taylor_step(x, h, y, yp);
    ai = y;
    aip = yp;
}

// Bi, Bi' at u in (0, kUAiry] by forward stepping from 0
__device__ inline void airy_bi_small(double u, double &bi, double &bip)
{
    // Bi(0) = 1 / (3^{1/6} Gamma(2/3)), Bi'(0) = 3^{1/6} / Gamma(1/3)
    double y = 0.61492662744600073515, yp = 0.44828835735382635791;
    const int steps = (int)ceil(u / kAiryStep);
    const double h = u / steps;
    double x = 0.0;
    for (int s = 0; s < steps; ++s, x += h) airy_taylor_step(x, h, y, yp);
    bi = y;
    bip = yp;
}

// T(u) = Ai'(u) Ci'(u) + u Ai(u) Ci(u), Ci = Ai - i Bi, for u > 0
__device__ inline void pp_term(double u, double &re, double &im)
{
    if (u > kUAiry) {
        const double zeta = (2.0 / 3.0) * u * sqrt(u);
        double sa, sap, sb, sbp;
        airy_asym_sums(zeta, sa, sap, sb, sbp);
        const double su = sqrt(u);
        re = su / (4.0 * M_PI) * exp(-2.0 * zeta) * (sap * sap + sa * sa);
        im = -su / (2.0 * M_PI) * (sa * sb - sap * sbp);
    } else {
        double ai, aip, bi, bip;
        airy_ai_small(u, ai, aip);
        airy_bi_small(u, bi, bip);
        re = aip * aip + u * ai * ai;
        im = -(aip * bip + u * ai * bi);
    }
}

// Hurwitz zeta(5, a), a >= 1/2, by Euler-Maclaurin summation from a + 8
__device__ inline double hurwitz_zeta5(double a)
{
    double s = 0.0;
    for (int k = 0; k < 8; ++k) {
        const double x = a + k;
        const double x2 = x * x;
        s += 1.0 / (x2 * x2 * x);
    }
    const double N = a + 8.0;
    const double iN = 1.0 / N, iN2 = iN * iN;
    double t = iN2 * iN2;                         // N^{-4}
    s += t / 4.0 + 0.5 * t * iN;                  // N^{1-s}/(s-1) + N^{-s}/2
    // sum_j B_{2j}/(2j)! (s)_{2j-1} N^{-s-2j+1}
    const double B[6] = {1.0 / 6.0, -1.0 / 30.0, 1.0 / 42.0, -1.0 / 30.0, 5.0 / 66.0, -691.0 / 2730.0};
    double poch = 5.0;                            // (5)_1
    double fact = 2.0;                            // (2j)!
    double pw = t * iN2;                          // N^{-6}
    for (int j = 1; j <= 6; ++j) {
        s += B[j - 1] / fact * poch * pw;
        poch *= (5.0 + 2 * j - 1) * (5.0 + 2 * j);
        fact *= (2.0 * j + 1.0) * (2.0 * j + 2.0);
        pw *= iN2;
    }
    return s;
}

__global__ __launch_bounds__(kThreads) void impedance_kernel(int nk, double dkappa, int model, double P,
                                                             double *__restrict__ zr, double *__restrict__ zi)
{
    const int k = blockIdx.x * kThreads + threadIdx.x;
    if (k >= nk) return;
    const double kap = k * dkappa;
    double re = 0.0, im = 0.0;
    if (k > 0 && model == VFP_Z_FREE_SPACE) {
        const double F = 0.9388929401017446;  // Gamma(2/3) / 3^{1/3}
        const double mag = F * cbrt(kap);
        re = mag * 0.86602540378443864676;          // cos 30deg
        im = mag * 0.5;
    } else if (k > 0 && model == VFP_Z_PARALLEL_PLATES) {
        const double A = M_PI * M_PI * exp2(-2.0 / 3.0) * P * P * pow(kap, -4.0 / 3.0);
        int pstar = 0;
        if (A <= kUAsym) pstar = (int)floor((sqrt(kUAsym / A) - 1.0) / 2.0) + 1;
        double sr = 0.0, si = 0.0;
        for (int p = 0; p < pstar; ++p) {
            const double q = 2.0 * p + 1.0;
            double tr, ti;
            pp_term(A * q * q, tr, ti);
            sr += tr;
            si += ti;
        }
        si += -(3.0 / (16.0 * M_PI)) * pow(A, -2.5) * hurwitz_zeta5(pstar + 0.5) / 32.0;
        const double pre = 4.0 * M_PI * M_PI * exp2(1.0 / 3.0) * P * pow(kap, -1.0 / 3.0);
        re = pre * sr;
        im = pre * si;
    }
    zr[k] = re;
    zi[k] = im;
}

}  // namespace vfp
