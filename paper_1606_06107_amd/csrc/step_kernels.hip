// Per-time-step kernels of the decoupled Hermite lattice Boltzmann scheme on
// D1Q7^D (D = 1, 2, 3) translational and D1Q7 rotational populations.
//
// One launch = one time step of Sec. V B of the paper, fused:
//   gather the streamed f(x, t) = f*(S(x - c_i), t-1)   (pull; S = wrap/clamp)
//   FP64 moments rho, rho u, E_t, e_r and the temperature T   (steps 3-4)
//   fourth-order Hermite equilibria f^eq(rho,u,T), g^eq(T)     (Sec. IV)
//   BGK relaxation of f; the post-collision f*(x, t) is stored in place of x
//   forward-Euler third-order-upwind advection of g with u, plus relaxation
//   (Sec. V A), g(x, t+1) stored
//   optional per-tile FP64 totals of time t (mass, momentum, energy)
// Populations are SoA [Q][N], node index x fastest.  Right after
// initialisation f is stored streamed (`streamed` = 1, read in place).
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "lbm_device.hpp"

namespace lbmx {

template <typename P> __device__ __forceinline__ const P *pop(const void *base, int i, uint32_t N) {
    return reinterpret_cast<const P *>(base) + (size_t)i * N;
}
template <typename P> __device__ __forceinline__ P *pop_w(void *base, int i, uint32_t N) {
    return reinterpret_cast<P *>(base) + (size_t)i * N;
}

// Fixed-order workgroup reduction of K doubles; thread 0 writes dst[0..K-1].
template <int NT, int K>
__device__ __forceinline__ void block_totals(double (&v)[K], double *dst) {
    __shared__ double red[NT / 64][K];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double s = wave_sum(v[k]);
        if (lane == 0) red[wv][k] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int w = 0; w < NT / 64; ++w) s += red[w][k];
            dst[k] = s;
        }
    }
}

// Rotational update g' = g - adv - omega (g - g^eq(T)), stored.  For FP32
// the relaxation increments r_j = omega (g^eq_j - g_j) are corrected so that
// sum_j r_j = omega (1 - sum g) and sum_j j^2 r_j = omega (T/r^2 - sum j^2 g)
// hold to FP64 rounding (see gfix_from_defects).
template <typename P>
__device__ __forceinline__ void rot_relax_store(const P (&gv)[7], const P (&adv)[7],
                                                const GeqCoef<P> &gc, P om, double omega,
                                                double T, double er, bool valid, void *g_out,
                                                uint32_t N, uint32_t node) {
    if constexpr (sizeof(P) == 4) {
        double s0 = 0.0, s2 = 0.0, g0 = 0.0;
        static_for<0, 7>([&](auto J) {
            constexpr int j = decltype(J)::value;
            const double rl = (double)(om * (geq_dir<P, j>(gc) - gv[j]));
            s0 += rl;
            g0 += (double)gv[j];
            if constexpr (j != 3) s2 += double((j - 3) * (j - 3)) * rl;
        });
        double al, ga;
        gfix_from_defects(omega * (1.0 - g0) - s0, omega * (T / (kR * kR) - er) - s2, al, ga);
        const P alp = (P)al, gam = (P)ga;
        static_for<0, 7>([&](auto J) {
            constexpr int j = decltype(J)::value;
            const P rl = om * (geq_dir<P, j>(gc) - gv[j]);
            const P fixj = P(kW1[iabs(j - 3)]) * (alp + P((j - 3) * (j - 3)) * gam);
            const P gn = gv[j] - adv[j] + (rl + fixj);
            if (valid) pop_w<P>(g_out, j, N)[node] = gn;
        });
    } else {
        static_for<0, 7>([&](auto J) {
            constexpr int j = decltype(J)::value;
            const P gn = gv[j] - adv[j] - om * (gv[j] - geq_dir<P, j>(gc));
            if (valid) pop_w<P>(g_out, j, N)[node] = gn;
        });
    }
}

// ---------------------------------------------------------------------------
// D = 1, 2: one node per thread, all Q populations in registers.
// ---------------------------------------------------------------------------
template <typename P, int D, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) k_step_12(StepArgs a) {
    constexpr int Q = Lat<D>::Q;
    constexpr int NT = TX * TY;
    const int tile = xcd_tile(blockIdx.x, a.ntiles);
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int x = (tile % a.tiles0) * TX + lx;
    const int y = (D >= 2) ? (tile / a.tiles0) * TY + ly : 0;
    const bool valid = x < a.n0 && (D < 2 || y < a.n1);
    const int xc = x < a.n0 ? x : a.n0 - 1;
    const int yc = (D >= 2) ? (y < a.n1 ? y : a.n1 - 1) : 0;
    const uint32_t N = a.N;
    const uint32_t node = (uint32_t)xc + (uint32_t)a.n0 * (uint32_t)yc;
    const int shift = 1 - a.streamed;

    // Streaming sources per axis (Sec. V: shift by the integer velocity).
    int sx[7], sy[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        sx[k] = nb_coord(xc, -(k - 3) * shift, a.n0, a.open0);
        sy[k] = (D >= 2) ? nb_coord(yc, -(k - 3) * shift, a.n1, a.open1) * a.n0 : 0;
    }

    P fv[Q];
    Mom M = {0.0, {0.0, 0.0, 0.0}, 0.0, 0.0};
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const uint32_t idx = (uint32_t)(sx[cx_of(i) + 3] + (D >= 2 ? sy[cy_of(i) + 3] : 0));
        fv[i] = pop<P>(a.f_in, i, N)[idx];
        const double v = (double)fv[i];
        M.m0 += v;
        if constexpr (cx_of(i) != 0) M.m1[0] += double(cx_of(i)) * v;
        if constexpr (D >= 2 && cy_of(i) != 0) M.m1[1] += double(cy_of(i)) * v;
        if constexpr (c2_of<D>(i) != 0) M.e2 += double(c2_of<D>(i)) * v;
    });
    P gv[7];
    static_for<0, 7>([&](auto J) {
        constexpr int j = decltype(J)::value;
        gv[j] = pop<P>(a.g_in, j, N)[node];
        if constexpr (j != 3) M.er += double((j - 3) * (j - 3)) * (double)gv[j];
    });

    double rho, u[3] = {0.0, 0.0, 0.0}, T, Etot;
    finish_moments<D>(M, a.n_rot, rho, u, T, Etot);

    if (a.partials) {  // uniform branch: totals of time t
        double tv[2 + D];
        tv[0] = valid ? rho : 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) tv[1 + d] = valid ? kR * M.m1[d] : 0.0;
        tv[1 + D] = valid ? Etot : 0.0;
        block_totals<NT, 2 + D>(tv, a.partials + (size_t)tile * (2 + D));
    }

    // BGK relaxation towards the Hermite equilibrium; store post-collision.
    const P up[3] = {(P)u[0], (P)u[1], (P)u[2]};
    const FeqCoef<P> fc = feq_coef<P, D>((P)rho, up, (P)T);
    const P om = (P)a.omega;
    if constexpr (sizeof(P) == 4) {
        // pass 1: FP64 sums of the FP32 increments (see fix_from_defects)
        double s0 = 0.0, s1[3] = {0.0, 0.0, 0.0}, s2 = 0.0;
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double dl = (double)(om * (feq_dir<P, D, i>(fc) - fv[i]));
            s0 += dl;
            if constexpr (cx_of(i) != 0) s1[0] += double(cx_of(i)) * dl;
            if constexpr (D >= 2 && cy_of(i) != 0) s1[1] += double(cy_of(i)) * dl;
            if constexpr (c2_of<D>(i) != 0) s2 += double(c2_of<D>(i)) * dl;
        });
        double mm = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) mm += M.m1[d] * M.m1[d];
        const double t2 = a.omega * (mm / rho + D * rho * T / (kR * kR) - M.e2);
        const double d1[3] = {-s1[0], -s1[1], -s1[2]};
        const Fix fx = fix_from_defects<D>(-s0, d1, t2 - s2);
        const P al = (P)fx.alpha, ga = (P)fx.gamma;
        const P be[3] = {(P)fx.beta[0], (P)fx.beta[1], (P)fx.beta[2]};
        // pass 2: same increments plus the correction
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const P dl = om * (feq_dir<P, D, i>(fc) - fv[i]);
            const P out = fv[i] + (dl + fix_dir<P, D, i>(al, be, ga));
            if (valid) pop_w<P>(a.f_out, i, N)[node] = out;
        });
    } else {
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const P fe = feq_dir<P, D, i>(fc);
            const P out = fv[i] - om * (fv[i] - fe);
            if (valid) pop_w<P>(a.f_out, i, N)[node] = out;
        });
    }

    // Rotational populations: upwind advection with u, relaxation to g^eq(T).
    int gx[5], gy[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        gx[k] = nb_coord(xc, k - 2, a.n0, a.open0) + a.n0 * yc;
        gy[k] = (D >= 2) ? xc + a.n0 * nb_coord(yc, k - 2, a.n1, a.open1) : 0;
    }
    const GeqCoef<P> gc = geq_coef<P>((P)T);
    const P nu0 = up[0] / P(kR), nu1 = up[1] / P(kR);
    P adv[7];
    static_for<0, 7>([&](auto J) {
        constexpr int j = decltype(J)::value;
        const P *gj = pop<P>(a.g_in, j, N);
        adv[j] = upwind3<P>(nu0, gj[gx[0]], gj[gx[1]], gv[j], gj[gx[3]], gj[gx[4]]);
        if constexpr (D >= 2) adv[j] += upwind3<P>(nu1, gj[gy[0]], gj[gy[1]], gv[j], gj[gy[3]], gj[gy[4]]);
    });
    rot_relax_store<P>(gv, adv, gc, om, a.omega, T, M.er, valid, a.g_out, N, node);
}

// ---------------------------------------------------------------------------
// D = 3: D3Q343 has too many populations for one thread's registers.  A
// workgroup of four waves serves 64 nodes; wave w owns a quarter of the
// populations (and two of the seven rotational ones).  Each wave accumulates
// partial FP64 moments of its populations, the partials meet in LDS and are
// summed in a fixed order, every wave derives the same rho, u, T, and then
// relaxes and stores the populations it holds in registers.
// ---------------------------------------------------------------------------
constexpr int kQ3 = 343;
constexpr int kSplit3 = 86;  // populations per wave: 86, 86, 86, 85

template <typename P, int W>
__device__ __forceinline__ void step3_wave(const StepArgs &a, const int (&sx)[7], const int (&sy)[7],
                                           const int (&sz)[7], uint32_t node, int xc, int yc,
                                           int zc, bool valid, int tile, double (*part)[64][6],
                                           double (*part2)[64][8]) {
    constexpr int LO = W * kSplit3;
    constexpr int HI = (W + 1) * kSplit3 < kQ3 ? (W + 1) * kSplit3 : kQ3;
    constexpr bool F32 = sizeof(P) == 4;
    const uint32_t N = a.N;
    const int lane = threadIdx.x & 63;
    P fv[HI - LO];
    double m0 = 0.0, mx = 0.0, my = 0.0, mz = 0.0, e2 = 0.0, er = 0.0;
    static_for<LO, HI>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const uint32_t idx = (uint32_t)(sx[cx_of(i) + 3] + sy[cy_of(i) + 3] + sz[cz_of(i) + 3]);
        const P f = pop<P>(a.f_in, i, N)[idx];
        fv[i - LO] = f;
        const double v = (double)f;
        m0 += v;
        if constexpr (cx_of(i) != 0) mx += double(cx_of(i)) * v;
        if constexpr (cy_of(i) != 0) my += double(cy_of(i)) * v;
        if constexpr (cz_of(i) != 0) mz += double(cz_of(i)) * v;
        if constexpr (c2_of<3>(i) != 0) e2 += double(c2_of<3>(i)) * v;
    });
    // rotational populations j = W and j = W + 4 (if < 7)
    constexpr int J0 = W, J1 = W + 4;
    constexpr bool HAS1 = J1 < 7;
    const P g0 = pop<P>(a.g_in, J0, N)[node];
    P g1 = P(0);
    if constexpr (HAS1) g1 = pop<P>(a.g_in, J1, N)[node];
    er += double((J0 - 3) * (J0 - 3)) * (double)g0;
    if constexpr (HAS1) er += double((J1 - 3) * (J1 - 3)) * (double)g1;

    part[W][lane][0] = m0;
    part[W][lane][1] = mx;
    part[W][lane][2] = my;
    part[W][lane][3] = mz;
    part[W][lane][4] = e2;
    part[W][lane][5] = er;
    __syncthreads();
    Mom M;
    M.m0 = part[0][lane][0] + part[1][lane][0] + part[2][lane][0] + part[3][lane][0];
    M.m1[0] = part[0][lane][1] + part[1][lane][1] + part[2][lane][1] + part[3][lane][1];
    M.m1[1] = part[0][lane][2] + part[1][lane][2] + part[2][lane][2] + part[3][lane][2];
    M.m1[2] = part[0][lane][3] + part[1][lane][3] + part[2][lane][3] + part[3][lane][3];
    M.e2 = part[0][lane][4] + part[1][lane][4] + part[2][lane][4] + part[3][lane][4];
    M.er = part[0][lane][5] + part[1][lane][5] + part[2][lane][5] + part[3][lane][5];
    double rho, u[3], T, Etot;
    finish_moments<3>(M, a.n_rot, rho, u, T, Etot);

    if constexpr (W == 0) {
        if (a.partials) {  // one wave holds all 64 nodes of the tile
            double t[5] = {valid ? rho : 0.0, valid ? kR * M.m1[0] : 0.0,
                           valid ? kR * M.m1[1] : 0.0, valid ? kR * M.m1[2] : 0.0,
                           valid ? Etot : 0.0};
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const double s = wave_sum(t[k]);
                if (lane == 0) a.partials[(size_t)tile * 5 + k] = s;
            }
        }
    }

    const P up[3] = {(P)u[0], (P)u[1], (P)u[2]};
    const FeqCoef<P> fc = feq_coef<P, 3>((P)rho, up, (P)T);
    const GeqCoef<P> gc = geq_coef<P>((P)T);
    const P om = (P)a.omega;

    // Rotational advection for the wave's j's: 3-D upwind stencil from global.
    const P nu[3] = {up[0] / P(kR), up[1] / P(kR), up[2] / P(kR)};
    const uint32_t sxy = (uint32_t)a.n0 * (uint32_t)a.n1;
    auto advect = [&](auto JJ, P gcen) -> P {
        constexpr int j = decltype(JJ)::value;
        const P *gj = pop<P>(a.g_in, j, N);
        P h[5];
        P adv = P(0);
#pragma unroll
        for (int k = 0; k < 5; ++k)
            h[k] = (k == 2) ? gcen : gj[nb_coord(xc, k - 2, a.n0, a.open0) + a.n0 * yc + sxy * zc];
        adv += upwind3<P>(nu[0], h[0], h[1], h[2], h[3], h[4]);
#pragma unroll
        for (int k = 0; k < 5; ++k)
            h[k] = (k == 2) ? gcen : gj[xc + a.n0 * nb_coord(yc, k - 2, a.n1, a.open1) + sxy * zc];
        adv += upwind3<P>(nu[1], h[0], h[1], h[2], h[3], h[4]);
#pragma unroll
        for (int k = 0; k < 5; ++k)
            h[k] = (k == 2) ? gcen : gj[xc + a.n0 * yc + sxy * nb_coord(zc, k - 2, a.n2, a.open2)];
        adv += upwind3<P>(nu[2], h[0], h[1], h[2], h[3], h[4]);
        return adv;
    };
    const P adv0 = advect(Int<J0>{}, g0);
    P adv1 = P(0);
    if constexpr (HAS1) adv1 = advect(Int<J1 < 7 ? J1 : 0>{}, g1);

    P al = P(0), ga = P(0), be[3] = {P(0), P(0), P(0)}, gal = P(0), gga = P(0);
    if constexpr (F32) {
        // FP64 sums of this wave's FP32 relaxation increments, combined over
        // the four waves in a fixed order (see fix_from_defects).
        double s0 = 0.0, s1x = 0.0, s1y = 0.0, s1z = 0.0, s2 = 0.0;
        static_for<LO, HI>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double dl = (double)(om * (feq_dir<P, 3, i>(fc) - fv[i - LO]));
            s0 += dl;
            if constexpr (cx_of(i) != 0) s1x += double(cx_of(i)) * dl;
            if constexpr (cy_of(i) != 0) s1y += double(cy_of(i)) * dl;
            if constexpr (cz_of(i) != 0) s1z += double(cz_of(i)) * dl;
            if constexpr (c2_of<3>(i) != 0) s2 += double(c2_of<3>(i)) * dl;
        });
        double rs0 = (double)(om * (geq_dir<P, J0>(gc) - g0));
        double rs2 = double((J0 - 3) * (J0 - 3)) * rs0;
        double gs = (double)g0;
        if constexpr (HAS1) {
            const double r1 = (double)(om * (geq_dir<P, J1 < 7 ? J1 : 0>(gc) - g1));
            rs0 += r1;
            rs2 += double((J1 - 3) * (J1 - 3)) * r1;
            gs += (double)g1;
        }
        part2[W][lane][0] = s0;
        part2[W][lane][1] = s1x;
        part2[W][lane][2] = s1y;
        part2[W][lane][3] = s1z;
        part2[W][lane][4] = s2;
        part2[W][lane][5] = rs0;
        part2[W][lane][6] = rs2;
        part2[W][lane][7] = gs;
        __syncthreads();
        double S[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            S[k] = part2[0][lane][k] + part2[1][lane][k] + part2[2][lane][k] + part2[3][lane][k];
        const double mm = M.m1[0] * M.m1[0] + M.m1[1] * M.m1[1] + M.m1[2] * M.m1[2];
        const double t2 = a.omega * (mm / rho + 3.0 * rho * T / (kR * kR) - M.e2);
        const double d1[3] = {-S[1], -S[2], -S[3]};
        const Fix fx = fix_from_defects<3>(-S[0], d1, t2 - S[4]);
        al = (P)fx.alpha;
        ga = (P)fx.gamma;
        be[0] = (P)fx.beta[0];
        be[1] = (P)fx.beta[1];
        be[2] = (P)fx.beta[2];
        double ga_d, ga_g;
        gfix_from_defects(a.omega * (1.0 - S[7]) - S[5], a.omega * (T / (kR * kR) - M.er) - S[6],
                          ga_d, ga_g);
        gal = (P)ga_d;
        gga = (P)ga_g;
    }
    static_for<LO, HI>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const P dl = om * (feq_dir<P, 3, i>(fc) - fv[i - LO]);
        P out;
        if constexpr (F32) out = fv[i - LO] + (dl + fix_dir<P, 3, i>(al, be, ga));
        else out = fv[i - LO] + dl;
        if (valid) pop_w<P>(a.f_out, i, N)[node] = out;
    });
    auto relax_store = [&](auto JJ, P gcen, P adv) {
        constexpr int j = decltype(JJ)::value;
        const P rl = om * (geq_dir<P, j>(gc) - gcen);
        P gn;
        if constexpr (F32)
            gn = gcen - adv + (rl + P(kW1[iabs(j - 3)]) * (gal + P((j - 3) * (j - 3)) * gga));
        else gn = gcen - adv + rl;
        if (valid) pop_w<P>(a.g_out, j, N)[node] = gn;
    };
    relax_store(Int<J0>{}, g0, adv0);
    if constexpr (HAS1) relax_store(Int<J1 < 7 ? J1 : 0>{}, g1, adv1);
}

template <typename P, int TX, int TY>
__global__ void __launch_bounds__(256) k_step_3(StepArgs a) {
    static_assert(TX * TY == 64, "64 nodes per workgroup");
    __shared__ double part[4][64][6];
    __shared__ double part2[4][64][8];
    const int tile = xcd_tile(blockIdx.x, a.ntiles);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int t0 = tile % a.tiles0, rest = tile / a.tiles0;
    const int t1 = rest % a.tiles1, t2 = rest / a.tiles1;
    const int x = t0 * TX + lane % TX, y = t1 * TY + lane / TX, z = t2;
    const bool valid = x < a.n0 && y < a.n1 && z < a.n2;
    const int xc = x < a.n0 ? x : a.n0 - 1, yc = y < a.n1 ? y : a.n1 - 1, zc = z;
    const uint32_t node = (uint32_t)xc + (uint32_t)a.n0 * ((uint32_t)yc + (uint32_t)a.n1 * zc);
    const int shift = 1 - a.streamed;
    int sx[7], sy[7], sz[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        sx[k] = nb_coord(xc, -(k - 3) * shift, a.n0, a.open0);
        sy[k] = nb_coord(yc, -(k - 3) * shift, a.n1, a.open1) * a.n0;
        sz[k] = nb_coord(zc, -(k - 3) * shift, a.n2, a.open2) * (a.n0 * a.n1);
    }
    switch (w) {  // wave-uniform
        case 0: step3_wave<P, 0>(a, sx, sy, sz, node, xc, yc, zc, valid, tile, part, part2); break;
        case 1: step3_wave<P, 1>(a, sx, sy, sz, node, xc, yc, zc, valid, tile, part, part2); break;
        case 2: step3_wave<P, 2>(a, sx, sy, sz, node, xc, yc, zc, valid, tile, part, part2); break;
        default: step3_wave<P, 3>(a, sx, sy, sz, node, xc, yc, zc, valid, tile, part, part2); break;
    }
}

// ---------------------------------------------------------------------------
// Initial state: f = f^eq(rho,u,T), g = g^eq(T), evaluated in FP64, stored
// streamed.
// ---------------------------------------------------------------------------
template <typename P, int D> __global__ void __launch_bounds__(256) k_init(InitArgs a) {
    const uint32_t x = blockIdx.x * 256u + threadIdx.x;
    if (x >= a.N) return;
    const double uu[3] = {a.u[x], D >= 2 ? a.u[(size_t)a.N + x] : 0.0,
                          D >= 3 ? a.u[2 * (size_t)a.N + x] : 0.0};
    const FeqCoef<double> fc = feq_coef<double, D>(a.rho[x], uu, a.T[x]);
    static_for<0, Lat<D>::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        pop_w<P>(a.f, i, a.N)[x] = (P)feq_dir<double, D, i>(fc);
    });
    const GeqCoef<double> gc = geq_coef<double>(a.T[x]);
    static_for<0, 7>([&](auto J) {
        constexpr int j = decltype(J)::value;
        pop_w<P>(a.g, j, a.N)[x] = (P)geq_dir<double, j>(gc);
    });
}

// ---------------------------------------------------------------------------
// Fields, totals and canonical export (runtime loop over populations).
// ---------------------------------------------------------------------------
template <int D> __device__ __forceinline__ uint32_t src_index(const FieldArgs &a, int x, int y, int z,
                                                              int i, int shift) {
    const int sx = nb_coord(x, -cx_of(i) * shift, a.n0, a.open0);
    const int sy = D >= 2 ? nb_coord(y, -cy_of(i) * shift, a.n1, a.open1) : 0;
    const int sz = D >= 3 ? nb_coord(z, -cz_of(i) * shift, a.n2, a.open2) : 0;
    return (uint32_t)sx + (uint32_t)a.n0 * ((uint32_t)sy + (uint32_t)a.n1 * (uint32_t)sz);
}

template <typename P, int D> __global__ void __launch_bounds__(256) k_fields(FieldArgs a) {
    const uint32_t x = blockIdx.x * 256u + threadIdx.x;
    const bool valid = x < a.N;
    const uint32_t xn = valid ? x : a.N - 1;
    const int cx = xn % a.n0, cy = (xn / a.n0) % a.n1, cz = xn / (a.n0 * a.n1);
    const int shift = 1 - a.streamed;
    Mom M = {0.0, {0.0, 0.0, 0.0}, 0.0, 0.0};
    for (int i = 0; i < Lat<D>::Q; ++i) {
        const double v = (double)pop<P>(a.f, i, a.N)[src_index<D>(a, cx, cy, cz, i, shift)];
        M.m0 += v;
        M.m1[0] += cx_of(i) * v;
        if (D >= 2) M.m1[1] += cy_of(i) * v;
        if (D >= 3) M.m1[2] += cz_of(i) * v;
        M.e2 += c2_of<D>(i) * v;
    }
    for (int j = 0; j < 7; ++j) M.er += double((j - 3) * (j - 3)) * (double)pop<P>(a.g, j, a.N)[xn];
    double rho, u[3] = {0.0, 0.0, 0.0}, T, Etot;
    finish_moments<D>(M, a.n_rot, rho, u, T, Etot);
    if (valid) {
        if (a.rho) a.rho[x] = rho;
        if (a.T) a.T[x] = T;
        if (a.u)
            for (int d = 0; d < D; ++d) a.u[(size_t)d * a.N + x] = u[d];
    }
    if (a.partials) {
        double tv[2 + D];
        tv[0] = valid ? rho : 0.0;
        for (int d = 0; d < D; ++d) tv[1 + d] = valid ? kR * M.m1[d] : 0.0;
        tv[1 + D] = valid ? Etot : 0.0;
        block_totals<256, 2 + D>(tv, a.partials + (size_t)blockIdx.x * (2 + D));
    }
}

template <typename P, int D> __global__ void __launch_bounds__(256) k_export(FieldArgs a) {
    const uint32_t x = blockIdx.x * 256u + threadIdx.x;
    if (x >= a.N) return;
    const int cx = x % a.n0, cy = (x / a.n0) % a.n1, cz = x / (a.n0 * a.n1);
    const int shift = 1 - a.streamed;
    if (a.f_out)
        for (int i = 0; i < Lat<D>::Q; ++i)
            pop_w<P>(a.f_out, i, a.N)[x] = pop<P>(a.f, i, a.N)[src_index<D>(a, cx, cy, cz, i, shift)];
    if (a.g_out)
        for (int j = 0; j < 7; ++j) pop_w<P>(a.g_out, j, a.N)[x] = pop<P>(a.g, j, a.N)[x];
}

__global__ void __launch_bounds__(256) k_reduce(const double *partials, int nparts, int K,
                                                double *out) {
    __shared__ double s[256];
    for (int k = 0; k < K; ++k) {
        double acc = 0.0;
        for (int p = threadIdx.x; p < nparts; p += 256) acc += partials[(size_t)p * K + k];
        s[threadIdx.x] = acc;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = s[0];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static unsigned blocks_for(uint32_t N) { return (N + 255u) / 256u; }

hipError_t launch_init(int dtype, int dim, const InitArgs &a, hipStream_t s) {
    const dim3 g(blocks_for(a.N)), b(256);
    if (dtype == 0) {
        if (dim == 1) hipLaunchKernelGGL((k_init<float, 1>), g, b, 0, s, a);
        else if (dim == 2) hipLaunchKernelGGL((k_init<float, 2>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_init<float, 3>), g, b, 0, s, a);
    } else {
        if (dim == 1) hipLaunchKernelGGL((k_init<double, 1>), g, b, 0, s, a);
        else if (dim == 2) hipLaunchKernelGGL((k_init<double, 2>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_init<double, 3>), g, b, 0, s, a);
    }
    return hipGetLastError();
}

int step_ntiles(int dim, const int tile[3], int n0, int n1, int n2, int *t0, int *t1, int *t2) {
    *t0 = (n0 + tile[0] - 1) / tile[0];
    *t1 = dim >= 2 ? (n1 + tile[1] - 1) / tile[1] : 1;
    *t2 = dim >= 3 ? n2 : 1;
    return *t0 * *t1 * *t2;
}

#define LBMX_TILES_1D(X) X(64, 1) X(128, 1) X(256, 1) X(512, 1) X(1024, 1)
#define LBMX_TILES_2D(X) X(64, 4) X(32, 8) X(128, 2) X(256, 1) X(64, 8) X(32, 16) X(16, 16) X(64, 2)
#define LBMX_TILES_3D(X) X(64, 1) X(32, 2) X(16, 4)

template <typename P> static hipError_t launch_step_t(int dim, const int tile[3], const StepArgs &a,
                                                      hipStream_t s) {
    const dim3 grid(a.ntiles);
    bool done = false;
#define L1(TXv, TYv)                                                                     \
    if (!done && dim == 1 && tile[0] == TXv && tile[1] == 1) {                           \
        hipLaunchKernelGGL((k_step_12<P, 1, TXv, 1>), grid, dim3(TXv), 0, s, a);         \
        done = true;                                                                     \
    }
#define L2(TXv, TYv)                                                                     \
    if (!done && dim == 2 && tile[0] == TXv && tile[1] == TYv) {                         \
        hipLaunchKernelGGL((k_step_12<P, 2, TXv, TYv>), grid, dim3(TXv * TYv), 0, s, a); \
        done = true;                                                                     \
    }
#define L3(TXv, TYv)                                                                     \
    if (!done && dim == 3 && tile[0] == TXv && tile[1] == TYv) {                         \
        hipLaunchKernelGGL((k_step_3<P, TXv, TYv>), grid, dim3(256), 0, s, a);           \
        done = true;                                                                     \
    }
    LBMX_TILES_1D(L1)
    LBMX_TILES_2D(L2)
    LBMX_TILES_3D(L3)
#undef L1
#undef L2
#undef L3
    if (!done) return hipErrorInvalidValue;
    return hipGetLastError();
}

bool step_tile_supported(int dtype, int dim, const int tile[3]) {
    (void)dtype;
    bool ok = false;
#define C1(TXv, TYv) ok = ok || (dim == 1 && tile[0] == TXv && tile[1] == 1 && tile[2] == 1);
#define C2(TXv, TYv) ok = ok || (dim == 2 && tile[0] == TXv && tile[1] == TYv && tile[2] == 1);
#define C3(TXv, TYv) ok = ok || (dim == 3 && tile[0] == TXv && tile[1] == TYv && tile[2] == 1);
    LBMX_TILES_1D(C1)
    LBMX_TILES_2D(C2)
    LBMX_TILES_3D(C3)
#undef C1
#undef C2
#undef C3
    return ok;
}

hipError_t launch_step(int dtype, int dim, const int tile[3], const StepArgs &a, hipStream_t s) {
    return dtype == 0 ? launch_step_t<float>(dim, tile, a, s) : launch_step_t<double>(dim, tile, a, s);
}

hipError_t launch_fields(int dtype, int dim, const FieldArgs &a, int *nblocks, hipStream_t s) {
    const dim3 g(blocks_for(a.N)), b(256);
    *nblocks = (int)g.x;
    if (dtype == 0) {
        if (dim == 1) hipLaunchKernelGGL((k_fields<float, 1>), g, b, 0, s, a);
        else if (dim == 2) hipLaunchKernelGGL((k_fields<float, 2>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_fields<float, 3>), g, b, 0, s, a);
    } else {
        if (dim == 1) hipLaunchKernelGGL((k_fields<double, 1>), g, b, 0, s, a);
        else if (dim == 2) hipLaunchKernelGGL((k_fields<double, 2>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_fields<double, 3>), g, b, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_export(int dtype, int dim, const FieldArgs &a, hipStream_t s) {
    const dim3 g(blocks_for(a.N)), b(256);
    if (dtype == 0) {
        if (dim == 1) hipLaunchKernelGGL((k_export<float, 1>), g, b, 0, s, a);
        else if (dim == 2) hipLaunchKernelGGL((k_export<float, 2>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_export<float, 3>), g, b, 0, s, a);
    } else {
        if (dim == 1) hipLaunchKernelGGL((k_export<double, 1>), g, b, 0, s, a);
        else if (dim == 2) hipLaunchKernelGGL((k_export<double, 2>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_export<double, 3>), g, b, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_reduce(const double *partials, int nparts, int K, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partials, nparts, K, out);
    return hipGetLastError();
}

}  // namespace lbmx
