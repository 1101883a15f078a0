// Per-time-step kernels of the decoupled Hermite lattice Boltzmann scheme on
// D1Q7^D (D = 1, 2, 3) translational and D1Q7 rotational populations.
//
// One launch = one time step of Sec. V B of the paper, fused:
//   gather the streamed f(x, t) = f*(S(x - c_i), t-1)   (pull; S = wrap/clamp)
//   FP64 moments rho, rho u, E_t, e_r and the temperature T   (steps 3-4)
//   fourth-order Hermite equilibria f^eq(rho,u,T), g^eq(T)     (Sec. IV)
//   BGK relaxation of f and its storage (below)
//   forward-Euler third-order-upwind advection of g with u, plus relaxation
//   (Sec. V A), g(x, t+1) stored
//   optional per-tile FP64 totals of time t (mass, momentum, energy)
// Populations are SoA [Q][N], node index x fastest.  Translational storage
// (kScheme* / kLayout* in launch.hpp): ping-pong (pull from f_in, the
// post-collision f*(x, t) stored at x in f_out) or, on grids periodic in
// every axis, in place in one buffer (even/odd steps).  The rotational
// populations always ping-pong.
//
// Ping-pong steps load f with the non-temporal hint and store with sc1 (the
// 470 MB working set streams through); in-place steps use the default policy
// (the single 206 MB f buffer at 1024^2 FP32 largely stays in the 256 MB
// memory-side cache).  Rotational stencil neighbours use cached loads.
//
// Kernel templates, included by the step_*.hip translation units that
// instantiate and launch them.
#pragma once
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

// Byte-addressed population access: non-temporal loads of f (each value is
// read once per step), cached loads of g (stencil neighbours are shared
// between nodes) and plain stores.
// `base` is uniform (population row), `off` the lane's 32-bit byte offset,
// which gives SGPR-base + VGPR-offset addressing.
template <typename P> __device__ __forceinline__ P ld_nt(const char *base, uint32_t off) {
    return __builtin_nontemporal_load(reinterpret_cast<const P *>(base + off));
}
template <typename P> __device__ __forceinline__ P ld(const char *base, uint32_t off) {
    return *reinterpret_cast<const P *>(base + off);
}
// Population stores: buffer form (explicit 32-bit lane offset) with the
// streaming cache policy; `i` selects the population row.
template <typename P> __device__ __forceinline__ void st(void *base, int i, uint32_t N,
                                                        uint32_t off, P v) {
    stp_stream<P>(base, i, N, off, v);
}

// Interior-wave form: buffer loads on a descriptor over population row `i`,
// at lane offset `vo` plus a uniform row offset `so` plus an immediate.
template <typename P, int CPOL>
__device__ __forceinline__ P ld_buf(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    if constexpr (sizeof(P) == 4)
        return __builtin_bit_cast(P, __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, CPOL));
    else
        return __builtin_bit_cast(P, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, CPOL));
}

// Lane shifts across the whole wave (DPP wave_shr:1 / wave_shl:1): lane l
// receives v from lane l-1 (SHR) or l+1 (SHL); the lane with no source
// (0, resp. 63) receives `fill`.  All 64 lanes must be active.
template <int CTRL>
__device__ __forceinline__ float wave_shift(float fill, float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, fill),
                                                                 __builtin_bit_cast(int, v), CTRL,
                                                                 0xF, 0xF, false));
}
constexpr int kWaveShr1 = 0x138, kWaveShl1 = 0x130;

template <typename P, int CPOL>
__device__ __forceinline__ void st_buf(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, P v) {
    if constexpr (sizeof(P) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)vo, (int)so, CPOL);
    else
        __builtin_amdgcn_raw_buffer_store_b64(
            __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v), r, (int)vo,
            (int)so, CPOL);
}
// A lane offset past every population row (N * sizeof(P) < 2^32): buffer
// stores to it are dropped by the range check.
constexpr uint32_t kDropOffset = 0xFFFFFFFFu;

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

// Rotational update g' = g - adv - omega (g - g^eq(T)), stored at byte
// offset `off`.  For FP32 the relaxation increments r_j = omega (g^eq_j - g_j)
// are corrected so that sum_j r_j = omega (1 - sum g) and
// sum_j j^2 r_j = omega (T/r^2 - sum j^2 g) hold to FP64 rounding (see
// gfix_from_defects).
template <typename P>
__device__ __forceinline__ void rot_relax_store(const P (&gv)[7], const P (&adv)[7],
                                                const GeqCoef<P> &gc, P om, double omega,
                                                double T, double er, void *g_out, uint32_t N,
                                                uint32_t off) {
    if constexpr (sizeof(P) == 4) {
        double s0 = 0.0, s2 = 0.0, g0 = 0.0;
        P rl[7];
        static_for<0, 7>([&](auto J) {
            constexpr int j = decltype(J)::value;
            rl[j] = om * (geq_dir<P, j>(gc) - gv[j]);
            s0 += (double)rl[j];
            g0 += (double)gv[j];
            if constexpr (j != 3) s2 += double((j - 3) * (j - 3)) * (double)rl[j];
        });
        double al, ga;
        gfix_from_defects(omega * (1.0 - g0) - s0, omega * (T * kInvR2 - er) - s2, al, ga);
        const P alp = (P)al, gam = (P)ga;
        static_for<0, 7>([&](auto J) {
            constexpr int j = decltype(J)::value;
            const P fixj = P(kW1[iabs(j - 3)]) * (alp + P((j - 3) * (j - 3)) * gam);
            stp_stream<P, kCpolStoreG>(g_out, j, N, off, gv[j] - adv[j] + (rl[j] + fixj));
        });
    } else {
        static_for<0, 7>([&](auto J) {
            constexpr int j = decltype(J)::value;
            stp_stream<P, kCpolStoreG>(g_out, j, N, off, gv[j] - adv[j] - om * (gv[j] - geq_dir<P, j>(gc)));
        });
    }
}

// ---------------------------------------------------------------------------
// D = 1, 2: one node per thread, all Q populations in registers.
// ---------------------------------------------------------------------------
// Waves per SIMD (min, max).  2-D FP32: exactly 3 -- measured on the 1024^2
// D2Q49 step, 3 concurrent waves per SIMD beat 4 by ~4 % (fewer interleaved
// DRAM streams, tighter L2 reuse of the rotational rows); the attribute pads
// the register allocation past the 4-wave limit.  Its tiles have at most 512
// threads (2 waves per SIMD per workgroup).  Otherwise at least 4 (FP32) or
// 2 (FP64) waves, i.e. at most 128 / 256 VGPRs.
template <typename P, int D> constexpr int kWavesMin = sizeof(P) == 4 ? (D == 2 ? 3 : 4) : 2;
template <typename P, int D> constexpr int kWavesMax = (sizeof(P) == 4 && D == 2) ? 3 : 8;

template <typename P, int D, int TX, int TY, int S, int K = kTensor>
__global__ void __launch_bounds__(TX *TY)
__attribute__((amdgpu_waves_per_eu(kWavesMin<P, D>, kWavesMax<P, D>))) k_step_12(StepArgs a) {
    static_assert(!(sizeof(P) == 4 && D == 2) || TX * TY <= 512, "3 waves per SIMD needs <= 512 threads");
    // Populations by storage slot i (0..Q-1), velocity c of direction
    // L::dir(i); slot Q-1-i holds -c, slot H the rest population.
    using L = Lat<D, K>;
    constexpr int Q = L::Q;
    constexpr int H = Q / 2;  // rest direction c = 0; pairs (i, Q-1-i) for i < H
    constexpr int NT = TX * TY;
    constexpr int NS = 2 * D + 1;  // populations absorbing the FP32 defects
    constexpr uint32_t SZ = sizeof(P);
    constexpr bool F32 = sizeof(P) == 4;

    const int tile = xcd_tile(blockIdx.x, a.ntiles, a.reverse);
    const int x0 = (tile % a.tiles0) * TX;
    const int y0 = D >= 2 ? (tile / a.tiles0) * TY : 0;
    const int lx = threadIdx.x % TX, ly = D >= 2 ? threadIdx.x / TX : 0;
    const int x = x0 + lx, y = y0 + ly;
    const bool valid = x < a.n0 && (D < 2 || y < a.n1);
    // Lanes past a ragged edge work on the clamped node: they load and
    // compute exactly what the lane of that node does.  Ping-pong stores of
    // theirs write the same bits to the same addresses and need no guard;
    // in-place translational stores of theirs are dropped (another wave may
    // not have read those locations yet).
    const int xc = x < a.n0 ? x : a.n0 - 1;
    const int yc = D >= 2 ? (y < a.n1 ? y : a.n1 - 1) : 0;
    const uint32_t N = a.N;
    const size_t PS = (size_t)N * SZ;             // bytes per population row
    const long RS = D >= 2 ? (long)a.n0 * SZ : 0;  // bytes per grid row
    const uint32_t nodeb = ((uint32_t)xc + (uint32_t)a.n0 * (uint32_t)yc) * SZ;
    const char *fin = static_cast<const char *>(a.f_in);
    const char *gin = static_cast<const char *>(a.g_in);
    // Interior waves (every lane's +-3 neighbourhood inside the grid, gather
    // from x - c): neighbour offsets are immediates (x) and uniform row
    // offsets (y).  Other waves wrap or clamp per lane.
    const bool inner = xc >= 3 && xc + 3 < a.n0 && (D < 2 || (yc >= 3 && yc + 3 < a.n1));
    const bool fast = (S != kSchemePingPong || a.layout == kLayoutPost) && __all(inner);

    // Interior lanes: vb = offset of (x-3, y-3) >= 0; row offsets in SGPRs.
    const uint32_t vb = nodeb - 3u * SZ - (D >= 2 ? 3u * (uint32_t)RS : 0u);
    uint32_t rowo[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) rowo[k] = D >= 2 ? (uint32_t)k * (uint32_t)RS : 0u;
    // In FP32 interior waves that cover 64 consecutive x, the x neighbours of
    // g come from adjacent lanes (DPP) plus four uniform halo values per j.
    constexpr bool XDPP = F32 && TX % 64 == 0;

    // 1. The streamed populations f_i(x, t): local (initial or even in-place
    //    step) or gathered from x - c_i, slot i (ping-pong) or slot opp(i)
    //    (odd in-place step).
    constexpr bool PP = S == kSchemePingPong;
    constexpr int CPL = PP ? kCpolLoadStream : 0;
    auto slot_in = [](int i) { return S == kSchemeInPlaceOdd ? Q - 1 - i : i; };
    P fv[Q];
    uint32_t sox[7], soy[7];  // scatter offsets of x + c (odd in-place step, edge waves)
    if constexpr (S == kSchemeInPlaceEven) {
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value, d = L::dir(i);
            fv[i] = ld_buf<P, 0>(pop_rsrc(a.f_in, i, N, SZ), nodeb, 0u);
        });
    } else {
        if (fast) {
            static_for<0, Q>([&](auto I) {
                constexpr int i = decltype(I)::value, d = L::dir(i);
                const __amdgpu_buffer_rsrc_t r = pop_rsrc(a.f_in, slot_in(i), N, SZ);
                fv[i] = ld_buf<P, CPL>(r, vb + (3 - cx_of(d)) * SZ, D >= 2 ? rowo[3 - cy_of(d)] : 0u);
            });
        } else {
            const int shift = (PP && a.layout == kLayoutStreamed) ? 0 : 1;
            uint32_t ox[7], oy[7];
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                ox[k] = (uint32_t)nb_coord(xc, -(k - 3) * shift, a.n0, a.open0) * SZ;
                oy[k] = D >= 2 ? (uint32_t)nb_coord(yc, -(k - 3) * shift, a.n1, a.open1) * (uint32_t)RS : 0u;
                if constexpr (S == kSchemeInPlaceOdd) {
                    sox[k] = (uint32_t)nb_coord(xc, k - 3, a.n0, 0) * SZ;
                    soy[k] = D >= 2 ? (uint32_t)nb_coord(yc, k - 3, a.n1, 0) * (uint32_t)RS : 0u;
                }
            }
            static_for<0, Q>([&](auto I) {
                constexpr int i = decltype(I)::value, d = L::dir(i);
                const uint32_t off = ox[cx_of(d) + 3] + (D >= 2 ? oy[cy_of(d) + 3] : 0u);
                if constexpr (PP) fv[i] = ld_nt<P>(fin + i * PS, off);
                else fv[i] = ld<P>(fin + slot_in(i) * PS, off);
            });
        }
    }
    // Translational store of direction i: ping-pong slot i at x (f_out);
    // even in-place slot opp(i) at x; odd in-place slot i at x + c_i.
    const uint32_t nodeb_st = valid ? nodeb : kDropOffset;
    auto store_f = [&](auto I, P v) {
        constexpr int i = decltype(I)::value, d = L::dir(i);
        if constexpr (PP) {
            st<P>(a.f_out, i, N, nodeb, v);
        } else if constexpr (S == kSchemeInPlaceEven) {
            st_buf<P, 0>(pop_rsrc(a.f_out, Q - 1 - i, N, SZ), nodeb_st, 0u, v);
        } else {
            const __amdgpu_buffer_rsrc_t r = pop_rsrc(a.f_out, i, N, SZ);
            if (fast)
                st_buf<P, 0>(r, vb + (3 + cx_of(d)) * SZ, D >= 2 ? rowo[3 + cy_of(d)] : 0u, v);
            else
                st_buf<P, 0>(r, valid ? sox[cx_of(d) + 3] + (D >= 2 ? soy[cy_of(d) + 3] : 0u) : kDropOffset,
                             0u, v);
        }
    };
    P gv[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) gv[j] = ld<P>(gin + j * PS, nodeb);

    // 2. FP64 moments via per-column (cx) and per-row (cy) sums.
    double col[7] = {0, 0, 0, 0, 0, 0, 0}, row[7] = {0, 0, 0, 0, 0, 0, 0};
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value, d = L::dir(i);
        const double v = (double)fv[i];
        col[cx_of(d) + 3] += v;
        if constexpr (D >= 2) row[cy_of(d) + 3] += v;
    });
    Mom M = {0.0, {0.0, 0.0, 0.0}, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        const double c = k - 3;
        M.m0 += col[k];
        M.m1[0] += c * col[k];
        M.e2 += c * c * col[k];
        if constexpr (D >= 2) {
            M.m1[1] += c * row[k];
            M.e2 += c * c * row[k];
        }
    }
#pragma unroll
    for (int j = 0; j < 7; ++j)
        if (j != 3) M.er += double((j - 3) * (j - 3)) * (double)gv[j];
    double rho, u[3] = {0.0, 0.0, 0.0}, T, Etot;
    const double inv = finish_moments<D>(M, a.n_rot, rho, u, T, Etot);

    if (a.partials) {  // uniform branch: totals of time t
        double tv[2 + D];
        tv[0] = valid ? rho : 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) tv[1 + d] = valid ? kR * M.m1[d] : 0.0;
        tv[1 + D] = valid ? Etot : 0.0;
        block_totals<NT, 2 + D>(tv, a.partials + (size_t)tile * (2 + D));
    }

    // 3. BGK relaxation towards the Hermite equilibrium; store post-collision.
    const P up[3] = {(P)u[0], (P)u[1], (P)u[2]};
    const P om = (P)a.omega;
    const FeqCoef<P> fc = feq_coef<P, D>((P)rho, up, (P)T);
    P dsp[NS];                               // increments of the special populations
    P cs[7] = {0, 0, 0, 0, 0, 0, 0}, rs[7] = {0, 0, 0, 0, 0, 0, 0};  // FP32 sums
    // Increment d = omega (f^eq - f), each use written as one multiply-add.
    auto relax = [&](auto I, P fe) {
        constexpr int i = decltype(I)::value, d = L::dir(i);
        constexpr int sr = special_rank<D>(d);
        const P df = fe - fv[i];
        if constexpr (F32) {
            cs[cx_of(d) + 3] += om * df;
            if constexpr (D >= 2) rs[cy_of(d) + 3] += om * df;
        }
        if constexpr (F32 && sr >= 0) dsp[sr] = om * df;
        else store_f(Int<i>{}, fv[i] + om * df);
    };
    static_for<0, H>([&](auto I) {
        constexpr int i = decltype(I)::value, k = Q - 1 - i, d = L::dir(i);
        P fp, fm;
        feq_pair<P, D, d, K>(fc, fp, fm);
        relax(Int<i>{}, fp);
        relax(Int<k>{}, fm);
    });
    relax(Int<H>{}, P(L::w(L::dir(H))) * fc.rho * fc.A0);
    if constexpr (F32) {
        double S0 = 0.0, S1[3] = {0.0, 0.0, 0.0}, S2 = 0.0;
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            const double c = k - 3, vc = (double)cs[k];
            S0 += vc;
            S1[0] += c * vc;
            S2 += c * c * vc;
            if constexpr (D >= 2) {
                const double vr = (double)rs[k];
                S1[1] += c * vr;
                S2 += c * c * vr;
            }
        }
        const double mm = M.m1[0] * M.m1[0] + (D >= 2 ? M.m1[1] * M.m1[1] : 0.0);
        const double t2 = a.omega * (mm * inv + D * rho * T * kInvR2 - M.e2);
        const double R1[3] = {-S1[0], -S1[1], 0.0};
        const Eps ep = eps_from_defects<D>(-S0, R1, t2 - S2);
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value, d = L::dir(i);
            constexpr int sr = special_rank<D>(d);
            if constexpr (sr >= 0) store_f(Int<i>{}, fv[i] + (dsp[sr] + (P)ep.e[sr]));
        });
    }

    // 4. Rotational populations: upwind advection with u, relaxation to
    //    g^eq(T).
    {
        const GeqCoef<P> gc = geq_coef<P>((P)T);
        const P nu0 = up[0] * P(1.0 / kR), nu1 = up[1] * P(1.0 / kR);
        P adv[7];
        P xdp[7], xdm[7], ydp[7], ydm[7];
        if (fast) {
            if constexpr (D >= 2) {
#pragma unroll
                for (int j = 0; j < 7; ++j) {
                    const __amdgpu_buffer_rsrc_t r = pop_rsrc(a.g_in, j, N, SZ);
                    upwind_diff<P>(ld_buf<P, 0>(r, vb + 3 * SZ, rowo[1]), ld_buf<P, 0>(r, vb + 3 * SZ, rowo[2]),
                                   gv[j], ld_buf<P, 0>(r, vb + 3 * SZ, rowo[4]),
                                   ld_buf<P, 0>(r, vb + 3 * SZ, rowo[5]), ydp[j], ydm[j]);
                }
            }
            if constexpr (XDPP) {
                const uint32_t wb = __builtin_amdgcn_readfirstlane(nodeb);  // lane 0's node
#pragma unroll
                for (int j = 0; j < 7; ++j) {
                    const P *gj = reinterpret_cast<const P *>(gin + j * PS + wb);
                    const P hm1 = wave_shift<kWaveShr1>(gj[-1], gv[j]);
                    const P hm2 = wave_shift<kWaveShr1>(gj[-2], hm1);
                    const P hp1 = wave_shift<kWaveShl1>(gj[64], gv[j]);
                    const P hp2 = wave_shift<kWaveShl1>(gj[65], hp1);
                    upwind_diff<P>(hm2, hm1, gv[j], hp1, hp2, xdp[j], xdm[j]);
                }
            } else {
#pragma unroll
                for (int j = 0; j < 7; ++j) {
                    const __amdgpu_buffer_rsrc_t r = pop_rsrc(a.g_in, j, N, SZ);
                    const uint32_t r3 = D >= 2 ? rowo[3] : 0u;
                    upwind_diff<P>(ld_buf<P, 0>(r, vb + 1 * SZ, r3), ld_buf<P, 0>(r, vb + 2 * SZ, r3), gv[j],
                                   ld_buf<P, 0>(r, vb + 4 * SZ, r3), ld_buf<P, 0>(r, vb + 5 * SZ, r3),
                                   xdp[j], xdm[j]);
                }
            }
        } else {
            uint32_t gxo[5], gyo[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                gxo[k] = ((uint32_t)nb_coord(xc, k - 2, a.n0, a.open0) + (uint32_t)a.n0 * (uint32_t)yc) * SZ;
                gyo[k] = D >= 2 ? ((uint32_t)xc + (uint32_t)a.n0 * (uint32_t)nb_coord(yc, k - 2, a.n1, a.open1)) * SZ
                                : 0u;
            }
#pragma unroll
            for (int j = 0; j < 7; ++j) {
                const char *gj = gin + j * PS;
                upwind_diff<P>(ld<P>(gj, gxo[0]), ld<P>(gj, gxo[1]), gv[j], ld<P>(gj, gxo[3]),
                               ld<P>(gj, gxo[4]), xdp[j], xdm[j]);
                if constexpr (D >= 2)
                    upwind_diff<P>(ld<P>(gj, gyo[0]), ld<P>(gj, gyo[1]), gv[j], ld<P>(gj, gyo[3]),
                                   ld<P>(gj, gyo[4]), ydp[j], ydm[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            adv[j] = upwind_apply<P>(nu0, xdp[j], xdm[j]);
            if constexpr (D >= 2) adv[j] += upwind_apply<P>(nu1, ydp[j], ydm[j]);
        }
        rot_relax_store<P>(gv, adv, gc, om, a.omega, T, M.er, a.g_out, N, nodeb);
    }

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

// Blocked value order (pop_index): the 64 nodes of a tile are one block, and
// the block of every source row starts at a uniform address.  Byte offsets:
struct Blk3 {
    uint32_t lo[7];        // lane's source within its row, per cx + 3
    size_t yb[7], zb[7];   // source row part, per cy + 3 and cz + 3
    size_t ob;             // the tile's own block
    uint32_t row_bytes;    // one row of blocks (n0 / 64 blocks)
};

template <typename P, int W, bool BLK>
__device__ __forceinline__ void step3_wave(const StepArgs &a, const int (&sx)[7], const int (&sy)[7],
                                           const int (&sz)[7], const Blk3 &B, uint32_t node, int xc,
                                           int yc, int zc, bool valid, int tile,
                                           double (*part)[64][6], double (*part2)[64][8]) {
    constexpr int LO = W * kSplit3;
    constexpr int HI = (W + 1) * kSplit3 < kQ3 ? (W + 1) * kSplit3 : kQ3;
    constexpr bool F32 = sizeof(P) == 4;
    const uint32_t N = a.N;
    const int lane = threadIdx.x & 63;
    P fv[HI - LO];
    double m0 = 0.0, mx = 0.0, my = 0.0, mz = 0.0, e2 = 0.0, er = 0.0;
    static_for<LO, HI>([&](auto I) {
        constexpr int i = decltype(I)::value;
        P f;
        if constexpr (BLK) {
            const char *row = reinterpret_cast<const char *>(a.f_in) + B.zb[cz_of(i) + 3] + B.yb[cy_of(i) + 3];
            const __amdgpu_buffer_rsrc_t r =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(row), 0, (int)B.row_bytes, kRsrcWord3);
            f = ld_buf<P, kCpolLoadStream>(r, B.lo[cx_of(i) + 3], (uint32_t)(i * kBlk * sizeof(P)));
        } else {
            const uint32_t idx = (uint32_t)(sx[cx_of(i) + 3] + sy[cy_of(i) + 3] + sz[cz_of(i) + 3]);
            f = ldp_stream<P>(a.f_in, i, N, idx * (uint32_t)sizeof(P));
        }
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
    const double inv = finish_moments<3>(M, a.n_rot, rho, u, T, Etot);

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
    const P nu[3] = {up[0] * P(1.0 / kR), up[1] * P(1.0 / kR), up[2] * P(1.0 / kR)};
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

    // BGK increments of this wave's populations; all but the special ones
    // (rest, +-e_a) are stored at once.  FP32: the increments' sums meet in
    // LDS and the defects go to the special populations (eps_from_defects).
    constexpr int NSP = 7;
    P dsp[NSP];
    __amdgpu_buffer_rsrc_t out_r;
    if constexpr (BLK)
        out_r = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<char *>(a.f_out) + B.ob, 0,
                                                  (int)(kQ3 * kBlk * sizeof(P)), kRsrcWord3);
    auto store_f = [&](int i, P v) {
        if constexpr (BLK)
            st_buf<P, kCpolStoreBlock>(out_r, (uint32_t)(lane * sizeof(P)), (uint32_t)(i * kBlk * sizeof(P)), v);
        else
            stp_stream<P>(a.f_out, i, N, node * (uint32_t)sizeof(P), v);
    };
    P s0 = P(0), s1x = P(0), s1y = P(0), s1z = P(0), s2 = P(0);
    static_for<LO, HI>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int sr = special_rank<3>(i);
        const P d = om * (feq_dir<P, 3, i>(fc) - fv[i - LO]);
        if constexpr (F32) {
            s0 += d;
            if constexpr (cx_of(i) != 0) s1x += P(cx_of(i)) * d;
            if constexpr (cy_of(i) != 0) s1y += P(cy_of(i)) * d;
            if constexpr (cz_of(i) != 0) s1z += P(cz_of(i)) * d;
            if constexpr (c2_of<3>(i) != 0) s2 += P(c2_of<3>(i)) * d;
        }
        if constexpr (F32 && sr >= 0) dsp[sr] = d;
        else if (valid) store_f(i, fv[i - LO] + d);
    });
    P gal = P(0), gga = P(0);
    if constexpr (F32) {
        double rs0 = (double)(om * (geq_dir<P, J0>(gc) - g0));
        double rs2 = double((J0 - 3) * (J0 - 3)) * rs0;
        double gs = (double)g0;
        if constexpr (HAS1) {
            const double r1 = (double)(om * (geq_dir<P, J1 < 7 ? J1 : 0>(gc) - g1));
            rs0 += r1;
            rs2 += double((J1 - 3) * (J1 - 3)) * r1;
            gs += (double)g1;
        }
        part2[W][lane][0] = (double)s0;
        part2[W][lane][1] = (double)s1x;
        part2[W][lane][2] = (double)s1y;
        part2[W][lane][3] = (double)s1z;
        part2[W][lane][4] = (double)s2;
        part2[W][lane][5] = rs0;
        part2[W][lane][6] = rs2;
        part2[W][lane][7] = gs;
        __syncthreads();
        double S[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            S[k] = part2[0][lane][k] + part2[1][lane][k] + part2[2][lane][k] + part2[3][lane][k];
        const double mm = M.m1[0] * M.m1[0] + M.m1[1] * M.m1[1] + M.m1[2] * M.m1[2];
        const double t2 = a.omega * (mm * inv + 3.0 * rho * T * kInvR2 - M.e2);
        const double R1[3] = {-S[1], -S[2], -S[3]};
        const Eps ep = eps_from_defects<3>(-S[0], R1, t2 - S[4]);
        static_for<LO, HI>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int sr = special_rank<3>(i);
            if constexpr (sr >= 0)
                if (valid) store_f(i, fv[i - LO] + (dsp[sr] + (P)ep.e[sr]));
        });
        double ga_d, ga_g;
        gfix_from_defects(a.omega * (1.0 - S[7]) - S[5], a.omega * (T * kInvR2 - M.er) - S[6],
                          ga_d, ga_g);
        gal = (P)ga_d;
        gga = (P)ga_g;
    }
    auto relax_store = [&](auto JJ, P gcen, P adv) {
        constexpr int j = decltype(JJ)::value;
        const P rl = om * (geq_dir<P, j>(gc) - gcen);
        P gn;
        if constexpr (F32)
            gn = gcen - adv + (rl + P(kW1[iabs(j - 3)]) * (gal + P((j - 3) * (j - 3)) * gga));
        else gn = gcen - adv + rl;
        if (valid) stp_stream<P, kCpolStoreG>(a.g_out, j, N, node * (uint32_t)sizeof(P), gn);
    };
    relax_store(Int<J0>{}, g0, adv0);
    if constexpr (HAS1) relax_store(Int<J1 < 7 ? J1 : 0>{}, g1, adv1);
}

template <typename P, int TX, int TY, bool BLK>
__global__ void __launch_bounds__(256) k_step_3(StepArgs a) {
    static_assert(!BLK || (TX == kBlk && TY == 1), "blocked order: one block per tile");
    static_assert(TX * TY == 64, "64 nodes per workgroup");
    __shared__ double part[4][64][6];
    __shared__ double part2[4][64][8];
    const int tile = xcd_tile(blockIdx.x, a.ntiles, a.reverse);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int t0 = tile % a.tiles0, rest = tile / a.tiles0;
    const int t1 = rest % a.tiles1, t2 = rest / a.tiles1;
    const int x = t0 * TX + lane % TX, y = t1 * TY + lane / TX, z = t2;
    const bool valid = x < a.n0 && y < a.n1 && z < a.n2;
    const int xc = x < a.n0 ? x : a.n0 - 1, yc = y < a.n1 ? y : a.n1 - 1, zc = z;
    const uint32_t node = (uint32_t)xc + (uint32_t)a.n0 * ((uint32_t)yc + (uint32_t)a.n1 * zc);
    const int shift = a.layout == kLayoutStreamed ? 0 : 1;
    int sx[7], sy[7], sz[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        sx[k] = nb_coord(xc, -(k - 3) * shift, a.n0, a.open0);
        sy[k] = nb_coord(yc, -(k - 3) * shift, a.n1, a.open1) * a.n0;
        sz[k] = nb_coord(zc, -(k - 3) * shift, a.n2, a.open2) * (a.n0 * a.n1);
    }
    Blk3 B;
    if constexpr (BLK) {  // n0 % 64 == 0: the tile is block t0 of row (y, z)
        const size_t blk_bytes = (size_t)kQ3 * kBlk * sizeof(P);
        const uint32_t tpr = (uint32_t)a.n0 / kBlk;
        B.row_bytes = (uint32_t)(tpr * blk_bytes);
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            const uint32_t xs = (uint32_t)sx[k];
            B.lo[k] = (uint32_t)((xs / kBlk) * blk_bytes + (xs % kBlk) * sizeof(P));
            B.yb[k] = (size_t)nb_coord(yc, -(k - 3) * shift, a.n1, a.open1) * B.row_bytes;
            B.zb[k] = (size_t)nb_coord(zc, -(k - 3) * shift, a.n2, a.open2) * a.n1 * B.row_bytes;
        }
        B.ob = ((size_t)t0 + (size_t)tpr * ((size_t)yc + (size_t)a.n1 * zc)) * blk_bytes;
    }
    switch (w) {  // wave-uniform
        case 0: step3_wave<P, 0, BLK>(a, sx, sy, sz, B, node, xc, yc, zc, valid, tile, part, part2); break;
        case 1: step3_wave<P, 1, BLK>(a, sx, sy, sz, B, node, xc, yc, zc, valid, tile, part, part2); break;
        case 2: step3_wave<P, 2, BLK>(a, sx, sy, sz, B, node, xc, yc, zc, valid, tile, part, part2); break;
        default: step3_wave<P, 3, BLK>(a, sx, sy, sz, B, node, xc, yc, zc, valid, tile, part, part2); break;
    }
}

// Launch k_step_12<P, D, tile, S> for a compiled tile shape; false if none.
template <typename P, int S>
bool launch_12(int dim, const int tile[3], const StepArgs &a, hipStream_t s) {
    const dim3 grid(a.ntiles);
    bool done = false;
#define L1(TXv, TYv)                                                                     \
    if (!done && dim == 1 && tile[0] == TXv) {                                           \
        hipLaunchKernelGGL((k_step_12<P, 1, TXv, 1, S>), grid, dim3(TXv), 0, s, a);       \
        done = true;                                                                     \
    }
#define L2(TXv, TYv)                                                                     \
    if (!done && dim == 2 && tile[0] == TXv && tile[1] == TYv) {                         \
        hipLaunchKernelGGL((k_step_12<P, 2, TXv, TYv, S>), grid, dim3(TXv * TYv), 0, s, a); \
        done = true;                                                                     \
    }
    LBMX_TILES_1D(L1)
    LBMX_TILES_2D(L2)
#undef L1
#undef L2
    return done;
}

// Launch k_step_12<P, 2, tile, S, kD2Q37> for a compiled D2Q37 tile shape.
template <typename P, int S>
bool launch_37(const int tile[3], const StepArgs &a, hipStream_t s) {
    const dim3 grid(a.ntiles);
    bool done = false;
#define L37(TXv, TYv)                                                                                 \
    if (!done && tile[0] == TXv && tile[1] == TYv) {                                                  \
        hipLaunchKernelGGL((k_step_12<P, 2, TXv, TYv, S, kD2Q37>), grid, dim3(TXv * TYv), 0, s, a); \
        done = true;                                                                                  \
    }
    LBMX_TILES_37(L37)
#undef L37
    return done;
}

}  // namespace lbmx
