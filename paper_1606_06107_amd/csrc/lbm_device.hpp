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

// D2Q37 (Table I): the D2Q49 velocities without the groups (2,2) and (3,2),
// one weight per group (p, q) = (max, min of |c_x|, |c_y|), at the same r.
constexpr double kW37[8] = {LBM_W37_0, LBM_W37_1, LBM_W37_2, LBM_W37_3,
                            LBM_W37_4, LBM_W37_5, LBM_W37_6, LBM_W37_7};
__host__ __device__ constexpr int d37_group(int i) {  // -1: not a D2Q37 velocity
    const int ax = iabs(cx_of(i)), ay = iabs(cy_of(i));
    const int p = ax > ay ? ax : ay, q = ax > ay ? ay : ax;
    if (p == 0) return 0;
    if (p == 1) return q == 0 ? 1 : 2;
    if (p == 2) return q == 0 ? 3 : (q == 1 ? 4 : -1);
    return q == 0 ? 5 : (q == 1 ? 6 : (q == 3 ? 7 : -1));
}

// Lattice kinds.  A population's storage slot s runs over 0..Q-1; its
// velocity is direction dir(s) of the base-7 enumeration above (the
// identity for the tensor lattices), so that slot Q-1-s holds -c.
enum { kTensor = 0, kD2Q37 = 1 };
template <int D, int K = kTensor> struct Lat {
    static constexpr int Q = D == 1 ? 7 : (D == 2 ? 49 : 343);
    __host__ __device__ static constexpr int dir(int s) { return s; }
    __host__ __device__ static constexpr double w(int d) { return w_of<D>(d); }
};
template <> struct Lat<2, kD2Q37> {
    static constexpr int Q = 37;
    __host__ __device__ static constexpr int dir(int s) {
        int k = 0;
        for (int i = 0; i < 49; ++i)
            if (d37_group(i) >= 0) {
                if (k == s) return i;
                ++k;
            }
        return -1;
    }
    __host__ __device__ static constexpr double w(int d) { return kW37[d37_group(d)]; }
};
// Slot -> direction as a table, for loops with a run-time slot index.
template <int D, int K> struct DirTable {
    int v[Lat<D, K>::Q];
    constexpr DirTable() : v() {
        for (int s = 0; s < Lat<D, K>::Q; ++s) v[s] = Lat<D, K>::dir(s);
    }
};

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

// 1/x for normal x to within about an ulp: the hardware estimate refined by
// two Newton-Raphson steps r <- r + r (1 - x r) (each squares the relative
// error).  A full IEEE division costs several times as many FP64 operations.
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

constexpr double kInvR2 = 1.0 / (kR * kR);

// Returns 1/rho.
template <int D> __device__ __forceinline__ double finish_moments(const Mom &M, double n_rot,
                                                                  double &rho, double u[3],
                                                                  double &T, double &Etot) {
    rho = M.m0;
    const double inv = rcp64(rho);
    double mm = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        u[a] = kR * M.m1[a] * inv;
        mm += M.m1[a] * M.m1[a];
    }
    const double Et = 0.5 * kR * kR * M.e2;
    const double rho_er = rho * 0.5 * n_rot * kR * kR * M.er;
    const double ke = 0.5 * kR * kR * mm * inv;
    T = 2.0 * rcp64(D + n_rot) * (Et + rho_er - ke) * inv;
    Etot = Et + rho_er;
    return inv;
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

template <typename P, int D, int I, int K = kTensor> __device__ __forceinline__ P feq_dir(const FeqCoef<P> &c) {
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
    return P(Lat<D, K>::w(I)) * c.rho * poly;
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
// Split form: the two one-sided differences do not depend on nu, so they can
// be formed as soon as the stencil values arrive.
template <typename P>
__device__ __forceinline__ void upwind_diff(P hm2, P hm1, P h0, P hp1, P hp2, P &dp, P &dm) {
    dp = (hm2 - P(6) * hm1 + P(3) * h0 + P(2) * hp1) * P(1.0 / 6.0);
    dm = (-hp2 + P(6) * hp1 - P(3) * h0 - P(2) * hm1) * P(1.0 / 6.0);
}
template <typename P> __device__ __forceinline__ P upwind_apply(P nu, P dp, P dm) {
    return nu * (nu >= P(0) ? dp : dm);
}
template <typename P> __device__ __forceinline__ P upwind3(P nu, P hm2, P hm1, P h0, P hp1, P hp2) {
    P dp, dm;
    upwind_diff<P>(hm2, hm1, h0, hp1, hp2, dp, dm);
    return upwind_apply<P>(nu, dp, dm);
}

// Periodic wrap or clamp of an arbitrary coordinate (tile halos may reach
// more than one period past the edge of a small grid).
__device__ __forceinline__ int wrap_any(int s, int n, int open) {
    if (open) return s < 0 ? 0 : (s >= n ? n - 1 : s);
    s %= n;
    return s < 0 ? s + n : s;
}

// Load/store population i at a 32-bit byte offset from the population's
// (uniform) base address: lets the compiler use SGPR-base + VGPR-offset
// addressing.  Requires N * sizeof(P) < 2^32.
template <typename P> __device__ __forceinline__ P ldp(const void *base, int i, uint32_t N,
                                                      uint32_t off) {
    const char *p = reinterpret_cast<const char *>(base) + (size_t)i * N * sizeof(P);
    return *reinterpret_cast<const P *>(p + off);
}
template <typename P> __device__ __forceinline__ void stp(void *base, int i, uint32_t N,
                                                         uint32_t off, P v) {
    char *p = reinterpret_cast<char *>(base) + (size_t)i * N * sizeof(P);
    *reinterpret_cast<P *>(p + off) = v;
}

// Streaming variants for the populations, which every time step reads once
// and writes once: loads carry the non-temporal hint and stores the sc1
// cache policy, issued as raw buffer operations on a descriptor spanning the
// population's row (out-of-range offsets read 0 / drop, never fault).  On
// gfx950 this pair keeps the ping-pong working set from thrashing L2 and the
// memory-side cache; measured on the pull pattern of a D2Q49 + D1Q7 step it
// is ~11 % faster than the default policy.
constexpr int kCpolLoadStream = 2;    // nt
constexpr int kCpolStoreStream = 16;  // sc1
// Rotational populations (always ping-pong) and the blocked 3-D stores, whose
// whole 87.8 kB block is written in one piece: sc1 + nt measured faster there.
constexpr int kCpolStoreG = 16;
constexpr int kCpolStoreBlock = 18;   // sc1 nt
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pop_rsrc(const void *base, int i, uint32_t N,
                                                           uint32_t sz) {
    const char *p = reinterpret_cast<const char *>(base) + (size_t)i * N * sz;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(p), 0, (int)(N * sz), kRsrcWord3);
}
template <typename P> __device__ __forceinline__ P ldp_stream(const void *base, int i, uint32_t N,
                                                             uint32_t off) {
    const __amdgpu_buffer_rsrc_t r = pop_rsrc(base, i, N, sizeof(P));
    if constexpr (sizeof(P) == 4)
        return __builtin_bit_cast(P, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, kCpolLoadStream));
    else
        return __builtin_bit_cast(P, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, kCpolLoadStream));
}
template <typename P, int CPOL = kCpolStoreStream>
__device__ __forceinline__ void stp_stream(void *base, int i, uint32_t N, uint32_t off, P v) {
    const __amdgpu_buffer_rsrc_t r = pop_rsrc(base, i, N, sizeof(P));
    if constexpr (sizeof(P) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0, CPOL);
    else
        __builtin_amdgcn_raw_buffer_store_b64(
            __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v), r,
            (int)off, 0, CPOL);
}

// Equilibrium of the direction pair (c, -c): with a = c.ru,
//   f^eq(+-c) / (w rho) = E(a^2) +- a O(a^2),  E = P0 + a^2 (P2 + a^2/24),
//   O = P1 + a^2/6   (same polynomial as feq_dir).
template <typename P, int D, int I, int K = kTensor>
__device__ __forceinline__ void feq_pair(const FeqCoef<P> &c, P &fplus, P &fminus) {
    constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I);
    constexpr double xi2d = kR * kR * c2_of<D>(I);
    const P xi2 = P(xi2d);
    P a = P(cx) * c.ru[0];
    if constexpr (D >= 2 && cy != 0) a += P(cy) * c.ru[1];
    if constexpr (D >= 3 && cz != 0) a += P(cz) * c.ru[2];
    const P a2 = a * a;
    const P p0 = c.A0 + xi2 * (c.A1 + xi2 * c.A2);
    const P p1 = c.B0 + xi2 * c.B1;
    const P p2 = c.C0 + xi2 * c.C1;
    const P E = p0 + a2 * (p2 + a2 * P(1.0 / 24.0));
    const P O = (p1 + a2 * P(1.0 / 6.0)) * a;
    const P wr = P(Lat<D, K>::w(I)) * c.rho;
    const P wE = wr * E;
    fplus = wE + wr * O;
    fminus = wE - wr * O;
}

// ---------------------------------------------------------------------------
// Conservative FP32 relaxation.  The BGK increments d_i = omega (f^eq_i - f_i)
// conserve mass and momentum and move sum_i |c_i|^2 f_i by
// t2 = omega (rho (|u|^2 + D T) / r^2 - e2) (integer-c units) in exact
// arithmetic.  In FP32 the rounded weights and polynomial bias these sums by
// ~1e-8 rho per step, which accumulates over thousands of steps.  The
// increments of all populations are summed; the defects
//   R0 = -sum d,  R1 = -sum c d,  R2 = t2 - sum |c|^2 d
// are then added to the 2D+1 populations with |c| <= 1 (rest and +-e_a),
// which are stored last:
//   eps_rest = R0 - R2,  eps_{+-e_a} = R2 / (2D) +- R1_a / 2,
// so the stored increments have exactly the target sums up to the final
// (unbiased) rounding of the stored values.  In exact arithmetic eps = 0.
// ---------------------------------------------------------------------------
template <int D> __host__ __device__ constexpr int special_rank(int i) {
    // 0 = rest, 1 + 2a = -e_a, 2 + 2a = +e_a, -1 = not special
    constexpr int H = Lat<D>::Q / 2;
    if (i == H) return 0;
    int p = 1;
    for (int a = 0; a < D; ++a, p *= 7) {
        if (i == H - p) return 1 + 2 * a;
        if (i == H + p) return 2 + 2 * a;
    }
    return -1;
}
struct Eps {
    double e[7];  // indexed by special_rank
};
template <int D> __device__ __forceinline__ Eps eps_from_defects(double R0, const double R1[3],
                                                                 double R2) {
    Eps x;
    x.e[0] = R0 - R2;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        constexpr double inv2d = 1.0 / (2.0 * D);
        x.e[1 + 2 * a] = a < D ? R2 * inv2d - 0.5 * R1[a] : 0.0;
        x.e[2 + 2 * a] = a < D ? R2 * inv2d + 0.5 * R1[a] : 0.0;
    }
    return x;
}

// Rotational analogue on D1Q7 with sum w j^2 = 1/r^2, sum w j^4 = 3/r^4:
// increment w_j (alpha + gamma j^2) removes the defects of sum_j and sum_j j^2.
__device__ __forceinline__ void gfix_from_defects(double d0, double d2, double &alpha,
                                                  double &gamma) {
    constexpr double r4h = 0.5 * kR * kR * kR * kR;
    gamma = (d2 - d0 * kInvR2) * r4h;
    alpha = d0 - gamma * kInvR2;
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
// halo rows through its own L2.  reverse = 1 walks every band from its far
// end.  Consecutive steps alternate the direction: a step then starts on
// the nodes its predecessor touched last, which are still in the
// memory-side cache (a working set about its size is otherwise swept in
// the order least favourable to it).
__device__ __forceinline__ int xcd_tile(int bid, int ntiles, int reverse) {
    const int q = ntiles >> 3, rem = ntiles & 7;
    const int xcd = bid & 7, k = bid >> 3;
    const int len = q + (xcd < rem ? 1 : 0);
    return xcd * q + (xcd < rem ? xcd : rem) + (reverse ? len - 1 - k : k);
}

// Deterministic wave64 sum (butterfly over fixed lane pairs).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace lbmx
