// Finite-difference time step of Sec. V A applied to both kinds of
// population (the alternative reading of the translational update):
//   f_i(x, t+dt) = f_i - sum_a (lambda c_ia) D_a[f_i] - (lambda/tau) (f_i - f_i^eq)
//   g_j(x, t+dt) = g_j - sum_a (lambda u_a / r) D_a[g_j] - (lambda/tau) (g_j - g_j^eq)
// with dt = lambda / r (lambda times the streaming step), D_a the third-order
// upwind difference along axis a oriented by the sign of the Courant number,
// and every term taken at time t (forward Euler).  One node per thread; the
// populations are read at their own node plus the three upwind neighbours per
// axis a population moves along; FP64 moments and temperature as in the
// streaming kernels.  Ping-pong between the two buffers; the values stay at
// their nodes, so the buffers always hold f(x, t) itself.
#include <hip/hip_runtime.h>

#include "fd.hpp"
#include "step_impl.hpp"

namespace lbmx {

template <typename P, int D, int K, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) k_step_fd(FdArgs a) {
    using L = Lat<D, K>;
    constexpr int Q = L::Q;
    constexpr int H = Q / 2;
    constexpr uint32_t SZ = sizeof(P);

    const int tile = xcd_tile(blockIdx.x, a.ntiles, 0);
    const int x0 = (tile % a.tiles0) * TX;
    const int y0 = D >= 2 ? (tile / a.tiles0) * TY : 0;
    const int x = x0 + (int)threadIdx.x % TX, y = y0 + (D >= 2 ? (int)threadIdx.x / TX : 0);
    // Lanes past a ragged edge compute the clamped node: same inputs, same
    // results, written to the same addresses (the buffers are distinct).
    const int xc = x < a.n0 ? x : a.n0 - 1;
    const int yc = D >= 2 ? (y < a.n1 ? y : a.n1 - 1) : 0;
    const uint32_t N = a.N;
    const size_t PS = (size_t)N * SZ;
    const uint32_t nodeb = ((uint32_t)xc + (uint32_t)a.n0 * (uint32_t)yc) * SZ;
    uint32_t ox[5], oy[5];  // byte offsets of the neighbours x-2..x+2, y-2..y+2
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        ox[k] = ((uint32_t)nb_coord(xc, k - 2, a.n0, a.open0) + (uint32_t)a.n0 * (uint32_t)yc) * SZ;
        oy[k] = D >= 2 ? ((uint32_t)xc + (uint32_t)a.n0 * (uint32_t)nb_coord(yc, k - 2, a.n1, a.open1)) * SZ
                       : nodeb;
    }
    const char *fin = static_cast<const char *>(a.f_in);
    const char *gin = static_cast<const char *>(a.g_in);

    // FP64 moments from per-column (c_x) and per-row (c_y) sums.  The
    // populations are not kept: each is read again (a cache hit) where it is
    // updated, which keeps the register count, and so the occupancy, of this
    // load-heavy kernel down (175 -> 113 registers in 2-D FP32).  Staging the
    // population planes through LDS measured slower than these cached reads.
    P gv[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) gv[j] = ld<P>(gin + j * PS, nodeb);
    double col[7] = {0, 0, 0, 0, 0, 0, 0}, row[7] = {0, 0, 0, 0, 0, 0, 0};
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value, d = L::dir(i);
        const double v = (double)ld<P>(fin + i * PS, nodeb);
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
    finish_moments<D>(M, a.n_rot, rho, u, T, Etot);

    const P up[3] = {(P)u[0], (P)u[1], (P)u[2]};
    const FeqCoef<P> fc = feq_coef<P, D>((P)rho, up, (P)T);
    const P lam = (P)a.lambda, om = (P)a.omega;

    // Translational populations: upwind advection with Courant number
    // lambda c_ia (only the upwind side of the stencil is read), relaxation.
    auto update = [&](auto I, P fe) {
        constexpr int i = decltype(I)::value, d = L::dir(i);
        constexpr int cx = cx_of(d), cy = cy_of(d);
        const char *fi = fin + i * PS;
        const P f0 = ld<P>(fi, nodeb);
        P adv = P(0);
        if constexpr (cx > 0)
            adv += (lam * P(cx)) * ((ld<P>(fi, ox[0]) - P(6) * ld<P>(fi, ox[1]) + P(3) * f0 +
                                     P(2) * ld<P>(fi, ox[3])) * P(1.0 / 6.0));
        if constexpr (cx < 0)
            adv += (lam * P(cx)) * ((-ld<P>(fi, ox[4]) + P(6) * ld<P>(fi, ox[3]) - P(3) * f0 -
                                     P(2) * ld<P>(fi, ox[1])) * P(1.0 / 6.0));
        if constexpr (D >= 2 && cy > 0)
            adv += (lam * P(cy)) * ((ld<P>(fi, oy[0]) - P(6) * ld<P>(fi, oy[1]) + P(3) * f0 +
                                     P(2) * ld<P>(fi, oy[3])) * P(1.0 / 6.0));
        if constexpr (D >= 2 && cy < 0)
            adv += (lam * P(cy)) * ((-ld<P>(fi, oy[4]) + P(6) * ld<P>(fi, oy[3]) - P(3) * f0 -
                                     P(2) * ld<P>(fi, oy[1])) * P(1.0 / 6.0));
        stp_stream<P>(a.f_out, i, N, nodeb, f0 - adv - om * (f0 - fe));
    };
    static_for<0, H>([&](auto I) {
        constexpr int i = decltype(I)::value, k = Q - 1 - i, d = L::dir(i);
        P fp, fm;
        feq_pair<P, D, d, K>(fc, fp, fm);
        update(Int<i>{}, fp);
        update(Int<k>{}, fm);
    });
    update(Int<H>{}, P(L::w(L::dir(H))) * fc.rho * fc.A0);

    // Rotational populations: upwind advection with lambda u / r, relaxation.
    const GeqCoef<P> gc = geq_coef<P>((P)T);
    const P nu0 = lam * up[0] * P(1.0 / kR), nu1 = lam * up[1] * P(1.0 / kR);
    P adv[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const char *gj = gin + j * PS;
        adv[j] = upwind3<P>(nu0, ld<P>(gj, ox[0]), ld<P>(gj, ox[1]), gv[j], ld<P>(gj, ox[3]), ld<P>(gj, ox[4]));
        if constexpr (D >= 2)
            adv[j] += upwind3<P>(nu1, ld<P>(gj, oy[0]), ld<P>(gj, oy[1]), gv[j], ld<P>(gj, oy[3]),
                                 ld<P>(gj, oy[4]));
    }
    rot_relax_store<P>(gv, adv, gc, om, a.omega, T, M.er, a.g_out, N, nodeb);
}

void fd_tile(int dim, int *tx, int *ty) {
    *tx = dim == 1 ? 256 : 64;
    *ty = dim == 1 ? 1 : 4;
}

hipError_t launch_step_fd(int dtype, int dim, int kind, const FdArgs &a, hipStream_t s) {
    const dim3 grid(a.ntiles);
    if (dim == 1 && kind == kTensor) {
        if (dtype == 0) hipLaunchKernelGGL((k_step_fd<float, 1, kTensor, 256, 1>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_step_fd<double, 1, kTensor, 256, 1>), grid, dim3(256), 0, s, a);
    } else if (dim == 2 && kind == kTensor) {
        if (dtype == 0) hipLaunchKernelGGL((k_step_fd<float, 2, kTensor, 64, 4>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_step_fd<double, 2, kTensor, 64, 4>), grid, dim3(256), 0, s, a);
    } else if (dim == 2 && kind == kD2Q37) {
        if (dtype == 0) hipLaunchKernelGGL((k_step_fd<float, 2, kD2Q37, 64, 4>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_step_fd<double, 2, kD2Q37, 64, 4>), grid, dim3(256), 0, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lbmx
