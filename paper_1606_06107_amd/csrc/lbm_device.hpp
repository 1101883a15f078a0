// Device-side arithmetic of the decoupled Hermite lattice Boltzmann scheme
// (Hu, Zhang & Geng, arXiv:1606.06107): lattice constants, FP64 moments and
// temperature, fourth-order Hermite equilibria, and the third-order upwind
// difference.  Shared by the per-step, batched and lifting kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice_constants.h"

namespace lbmx {

// ---------------------------------------------------------------------------
// Lattice (Table II; tensor powers D1Q7^D).  Direction i -> c = (cx, cy, cz)
// from the base-7 digits of i minus 3; w_i = w1(|cx|) w1(|cy|) w1(|cz|).
// ---------------------------------------------------------------------------
constexpr double kR = LBM_R;
constexpr double kW1[4] = {LBM_W1_0, LBM_W1_1, LBM_W1_2, LBM_W1_3};

template <int D> struct Lat {
    static constexpr int Q = D == 1 ? 7 : (D == 2 ? 49 : 343);
};
__host__ __device__ constexpr int cx_of(int i) { return i % 7 - 3; }
__host__ __device__ constexpr int cy_of(int i) { return (i / 7) % 7 - 3; }
__host__ __device__ constexpr int cz_of(int i) { return (i / 49) % 7 - 3; }
__host__ __device__ constexpr int iabs(int v) { return v < 0 ? -v : v; }
template <int D> __host__ __device__ constexpr int c2_of(int i) {
    return cx_of(i) * cx_of(i) + (D >= 2 ? cy_of(i) * cy_of(i) : 0) +
           (D >= 3 ? cz_of(i) * cz_of(i) : 0);
}
template <int D> __host__ __device__ constexpr double w_of(int i) {
    return kW1[iabs(cx_of(i))] * (D >= 2 ? kW1[iabs(cy_of(i))] : 1.0) *
           (D >= 3 ? kW1[iabs(cz_of(i))] : 1.0);
}

// Compile-time loop: calls f(std::integral_constant-like) for I = B..E-1.
template <int I> struct Int { static constexpr int value = I; };
template <int B, int E, typename F> __device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(Int<B>{});
        static_for<B + 1, E>(f);
    }
}

// ---------------------------------------------------------------------------
// Moments (Sec. V B steps 3-4), accumulated in FP64 whatever the population
// type.  In integer lattice units: m0 = sum f, m[a] = sum f c_a,
// e2 = sum f |c|^2, er = sum_j j^2 g_j.  Then
//   rho = m0, u = r m / rho, E_t = r^2 e2 / 2, e_r = (n/2) r^2 er,
//   T = 2/(D+n) (E_t + rho e_r - rho |u|^2 / 2) / rho.
// ---------------------------------------------------------------------------
struct Mom {
    double m0, m1[3], e2, er;
};

template <int D> __device__ __forceinline__ void finish_moments(const Mom &M, double n_rot,
                                                                double &rho, double u[3],
                                                                double &T, double &Etot) {
    rho = M.m0;
    const double inv = 1.0 / rho;
    double mm = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        u[a] = kR * M.m1[a] * inv;
        mm += M.m1[a] * M.m1[a];
    }
    const double Et = 0.5 * kR * kR * M.e2;
    const double rho_er = rho * 0.5 * n_rot * kR * kR * M.er;
    const double ke = 0.5 * kR * kR * mm * inv;
    T = 2.0 / (D + n_rot) * (Et + rho_er - ke) * inv;
    Etot = Et + rho_er;
}

// ---------------------------------------------------------------------------
// Translational equilibrium (Sec. IV): w rho sum_{k<=4} a^(k).H^(k)(xi) / k!
// for a Maxwellian of velocity u and temperature theta, written as a
// polynomial in a = xi.u with coefficients polynomial in |xi|^2:
//   f^eq / (w rho) = P0 + a (P1 + a (P2 + a (1/6 + a/24)))
//   P0 = A0 + xi2 (A1 + xi2 A2),  P1 = B0 + xi2 B1,  P2 = C0 + xi2 C1.
// ---------------------------------------------------------------------------
template <typename P> struct FeqCoef {
    P A0, A1, A2, B0, B1, C0, C1;
    P rho, ru[3];  // ru = r u (so that a = c . ru for integer c)
};

template <typename P, int D> __device__ __forceinline__ FeqCoef<P> feq_coef(P rho, const P u[3],
                                                                           P theta) {
    FeqCoef<P> c;
    P u2 = P(0);
#pragma unroll
    for (int a = 0; a < D; ++a) u2 += u[a] * u[a];
    const P t1 = theta - P(1);
    const P Dp = P(D);
    c.A0 = P(1) - P(0.5) * u2 - P(0.5) * Dp * t1 + P(0.125) * u2 * u2 +
           P(0.25) * (Dp + P(2)) * t1 * u2 + P(0.125) * Dp * (Dp + P(2)) * t1 * t1;
    c.A1 = P(0.5) * t1 - P(0.25) * t1 * u2 - P(0.25) * (Dp + P(2)) * t1 * t1;
    c.A2 = P(0.125) * t1 * t1;
    c.B0 = P(1) - P(0.5) * u2 - P(0.5) * (Dp + P(2)) * t1;
    c.B1 = P(0.5) * t1;
    c.C0 = P(0.5) - P(0.25) * u2 - P(0.25) * (Dp + P(4)) * t1;
    c.C1 = P(0.25) * t1;
    c.rho = rho;
#pragma unroll
    for (int a = 0; a < 3; ++a) c.ru[a] = a < D ? P(kR) * u[a] : P(0);
    return c;
}

template <typename P, int D, int I> __device__ __forceinline__ P feq_dir(const FeqCoef<P> &c) {
    constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I);
    constexpr double xi2d = kR * kR * c2_of<D>(I);
    const P xi2 = P(xi2d);
    P a = P(cx) * c.ru[0];
    if constexpr (D >= 2) a += P(cy) * c.ru[1];
    if constexpr (D >= 3) a += P(cz) * c.ru[2];
    const P p0 = c.A0 + xi2 * (c.A1 + xi2 * c.A2);
    const P p1 = c.B0 + xi2 * c.B1;
    const P p2 = c.C0 + xi2 * c.C1;
    const P poly = p0 + a * (p1 + a * (p2 + a * (P(1.0 / 6.0) + a * P(1.0 / 24.0))));
    return P(w_of<D>(I)) * c.rho * poly;
}

// ---------------------------------------------------------------------------
// Rotational equilibrium (Sec. IV): 1-D fourth-order Hermite expansion of a
// zero-mean Gaussian of variance theta:
//   g^eq_j = w_j [1 + (theta-1)(eta^2-1)/2 + (theta-1)^2 (eta^4 - 6 eta^2 + 3)/8]
// = w_j (G0 + eta^2 (G1 + eta^2 G2)).
// ---------------------------------------------------------------------------
template <typename P> struct GeqCoef {
    P G0, G1, G2;
};
template <typename P> __device__ __forceinline__ GeqCoef<P> geq_coef(P theta) {
    const P t1 = theta - P(1);
    GeqCoef<P> c;
    c.G0 = P(1) - P(0.5) * t1 + P(0.375) * t1 * t1;
    c.G1 = P(0.5) * t1 - P(0.75) * t1 * t1;
    c.G2 = P(0.125) * t1 * t1;
    return c;
}
template <typename P, int J> __device__ __forceinline__ P geq_dir(const GeqCoef<P> &c) {
    constexpr double e2 = kR * kR * (J - 3) * (J - 3);
    return P(kW1[iabs(J - 3)]) * (c.G0 + P(e2) * (c.G1 + P(e2) * c.G2));
}

// ---------------------------------------------------------------------------
// Third-order upwind difference of Sec. V A, times the Courant number nu:
//   nu >= 0: nu (h[-2] - 6 h[-1] + 3 h[0] + 2 h[+1]) / 6
//   nu <  0: nu (-h[+2] + 6 h[+1] - 3 h[0] - 2 h[-1]) / 6
// ---------------------------------------------------------------------------
template <typename P> __device__ __forceinline__ P upwind3(P nu, P hm2, P hm1, P h0, P hp1, P hp2) {
    const P dp = (hm2 - P(6) * hm1 + P(3) * h0 + P(2) * hp1) / P(6);
    const P dm = (-hp2 + P(6) * hp1 - P(3) * h0 - P(2) * hm1) / P(6);
    return nu * (nu >= P(0) ? dp : dm);
}

// ---------------------------------------------------------------------------
// Conservative FP32 relaxation.  The BGK increment d_i = omega (f^eq_i - f_i)
// conserves mass and momentum and moves sum_i |c_i|^2 f_i by
// omega (rho (|u|^2 + D T) / r^2 - e2) (integer-c units) in exact
// arithmetic.  In FP32 the rounded weights and polynomial bias these sums by
// ~1e-8 per step, which accumulates over thousands of steps.  The sums of
// the FP32 increments are taken in FP64 and the defects (d0, d1, d2) are
// removed with the increment w_i (alpha + beta.c_i + gamma |c_i|^2), using
// the lattice moments sum w = 1, sum w c_a c_b = delta_ab / r^2,
// sum w |c|^4 = D (D+2) / r^4.  In exact arithmetic the defects are zero.
// ---------------------------------------------------------------------------
struct Fix {
    double alpha, beta[3], gamma;
};
template <int D> __device__ __forceinline__ Fix fix_from_defects(double d0, const double d1[3],
                                                                 double d2) {
    constexpr double r2 = kR * kR;
    Fix x;
    x.gamma = (d2 - d0 * D / r2) * r2 * r2 / (2.0 * D);
    x.alpha = d0 - x.gamma * D / r2;
#pragma unroll
    for (int a = 0; a < 3; ++a) x.beta[a] = a < D ? r2 * d1[a] : 0.0;
    return x;
}
template <typename P, int D, int I> __device__ __forceinline__ P fix_dir(P alpha, const P beta[3],
                                                                        P gamma) {
    P v = alpha + P(c2_of<D>(I)) * gamma;
    if constexpr (cx_of(I) != 0) v += P(cx_of(I)) * beta[0];
    if constexpr (D >= 2 && cy_of(I) != 0) v += P(cy_of(I)) * beta[1];
    if constexpr (D >= 3 && cz_of(I) != 0) v += P(cz_of(I)) * beta[2];
    return P(w_of<D>(I)) * v;
}
// Rotational analogue on D1Q7 with sum w j^2 = 1/r^2, sum w j^4 = 3/r^4:
// increment w_j (alpha + gamma j^2) removes the defects of sum_j and sum_j j^2.
__device__ __forceinline__ void gfix_from_defects(double d0, double d2, double &alpha,
                                                  double &gamma) {
    constexpr double r2 = kR * kR;
    gamma = (d2 - d0 / r2) * r2 * r2 / 2.0;
    alpha = d0 - gamma / r2;
}

// Neighbour coordinate along one axis: periodic wrap (n >= 3, |d| <= 3) or
// clamp to [0, n-1] (open boundary).
__device__ __forceinline__ int nb_coord(int x, int d, int n, int open) {
    int s = x + d;
    if (open) return s < 0 ? 0 : (s >= n ? n - 1 : s);
    s += (s < 0) ? n : 0;
    s -= (s >= n) ? n : 0;
    return s;
}

// Map a workgroup id to a tile id so that each of the 8 XCDs (which receive
// workgroups round-robin) works on one contiguous band of tiles and shares
// halo rows through its own L2.
__device__ __forceinline__ int xcd_tile(int bid, int ntiles) {
    const int q = ntiles >> 3, rem = ntiles & 7;
    const int xcd = bid & 7, k = bid >> 3;
    return xcd * q + (xcd < rem ? xcd : rem) + k;
}

// Deterministic wave64 sum (butterfly over fixed lane pairs).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace lbmx
