// Initialisation, field/total extraction, canonical export and the
// fixed-order reduction; plus the step-launch dispatcher.
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
// Translational slot i of node x in either value order.
template <typename P, int D, int K>
__device__ __forceinline__ P fget(const void *base, int blocked, uint32_t N, int i, uint32_t x) {
    return reinterpret_cast<const P *>(base)[pop_index(blocked, Lat<D, K>::Q, N, i, x)];
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

// ---------------------------------------------------------------------------
// Initial state: f = f^eq(rho,u,T), g = g^eq(T), evaluated in FP64, stored
// streamed (kLayoutStreamed).
// ---------------------------------------------------------------------------
template <typename P, int D, int K> __global__ void __launch_bounds__(256) k_init(InitArgs a) {
    using L = Lat<D, K>;
    const uint32_t x = blockIdx.x * 256u + threadIdx.x;
    if (x >= a.N) return;
    const double uu[3] = {a.u[x], D >= 2 ? a.u[(size_t)a.N + x] : 0.0,
                          D >= 3 ? a.u[2 * (size_t)a.N + x] : 0.0};
    const FeqCoef<double> fc = feq_coef<double, D>(a.rho[x], uu, a.T[x]);
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        reinterpret_cast<P *>(a.f)[pop_index(a.blocked, L::Q, a.N, i, x)] =
            (P)feq_dir<double, D, L::dir(i), K>(fc);
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
// Node holding the value of f_i(x, t) for the buffer's layout (its slot is
// src_slot); d = the direction of slot i.
template <int D, int K> __device__ __forceinline__ int src_slot(const FieldArgs &a, int i) {
    return a.layout == kLayoutSwapped ? Lat<D, K>::Q - 1 - i : i;
}
template <int D> __device__ __forceinline__ uint32_t src_index(const FieldArgs &a, int x, int y, int z,
                                                              int d, int shift) {
    const int sx = nb_coord(x, -cx_of(d) * shift, a.n0, a.open0);
    const int sy = D >= 2 ? nb_coord(y, -cy_of(d) * shift, a.n1, a.open1) : 0;
    const int sz = D >= 3 ? nb_coord(z, -cz_of(d) * shift, a.n2, a.open2) : 0;
    return (uint32_t)sx + (uint32_t)a.n0 * ((uint32_t)sy + (uint32_t)a.n1 * (uint32_t)sz);
}

template <typename P, int D, int K> __global__ void __launch_bounds__(256) k_fields(FieldArgs a) {
    using L = Lat<D, K>;
    constexpr DirTable<D, K> dirs;
    const uint32_t x = blockIdx.x * 256u + threadIdx.x;
    const bool valid = x < a.N;
    const uint32_t xn = valid ? x : a.N - 1;
    const int cx = xn % a.n0, cy = (xn / a.n0) % a.n1, cz = xn / (a.n0 * a.n1);
    const int shift = a.layout == kLayoutStreamed ? 0 : 1;
    Mom M = {0.0, {0.0, 0.0, 0.0}, 0.0, 0.0};
    for (int i = 0; i < L::Q; ++i) {
        const int d = dirs.v[i];
        const double v = (double)fget<P, D, K>(a.f, a.blocked, a.N, src_slot<D, K>(a, i),
                                               src_index<D>(a, cx, cy, cz, d, shift));
        M.m0 += v;
        M.m1[0] += cx_of(d) * v;
        if (D >= 2) M.m1[1] += cy_of(d) * v;
        if (D >= 3) M.m1[2] += cz_of(d) * v;
        M.e2 += c2_of<D>(d) * v;
    }
    for (int j = 0; j < 7; ++j) M.er += double((j - 3) * (j - 3)) * (double)pop<P>(a.g, j, a.N)[xn];
    double n_rot = a.n_rot;
    if (a.offsets) {  // packed batch: binary search for the node's tube
        int lo = 0, hi = a.num_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.offsets[mid] <= (int64_t)xn) lo = mid;
            else hi = mid - 1;
        }
        n_rot = a.n_rot_inst[lo];
    }
    double rho, u[3] = {0.0, 0.0, 0.0}, T, Etot;
    finish_moments<D>(M, n_rot, rho, u, T, Etot);
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

template <typename P, int D, int K> __global__ void __launch_bounds__(256) k_export(FieldArgs a) {
    using L = Lat<D, K>;
    constexpr DirTable<D, K> dirs;
    const uint32_t x = blockIdx.x * 256u + threadIdx.x;
    if (x >= a.N) return;
    const int cx = x % a.n0, cy = (x / a.n0) % a.n1, cz = x / (a.n0 * a.n1);
    const int shift = a.layout == kLayoutStreamed ? 0 : 1;
    if (a.f_out)
        for (int i = 0; i < L::Q; ++i)
            pop_w<P>(a.f_out, i, a.N)[x] = fget<P, D, K>(a.f, a.blocked, a.N, src_slot<D, K>(a, i),
                                                         src_index<D>(a, cx, cy, cz, dirs.v[i], shift));
    if (a.g_out)
        for (int j = 0; j < 7; ++j) pop_w<P>(a.g_out, j, a.N)[x] = pop<P>(a.g, j, a.N)[x];
}

static unsigned blocks_for(uint32_t N);

// ---------------------------------------------------------------------------
// Rotational advection in m sub-steps (lbm_desc.g_substeps = m > 1): a plain
// one-node-per-thread path, ping-pong only.  One time step is
//   f*_i(x) = f_i - omega (f_i - f^eq_i)   (post-collision, pulled next step)
//   g(t+1)  = A^m g(t) - omega (g(t) - g^eq(T))
// with A the forward-Euler third-order upwind advection of Sec. V A at
// Courant numbers u_a / (m r), u from the moments of time t.  m = 1 would be
// the paper's update (the fused step kernels run that).
// ---------------------------------------------------------------------------
// f^eq of direction d (runtime) from the coefficients of feq_coef: the
// polynomial of feq_dir.
template <typename P, int D, int K> __device__ __forceinline__ P feq_rt(const FeqCoef<P> &c, int d) {
    const P xi2 = P(kR * kR * c2_of<D>(d));
    P a = P(cx_of(d)) * c.ru[0];
    if (D >= 2) a += P(cy_of(d)) * c.ru[1];
    if (D >= 3) a += P(cz_of(d)) * c.ru[2];
    const P p0 = c.A0 + xi2 * (c.A1 + xi2 * c.A2);
    const P p1 = c.B0 + xi2 * c.B1;
    const P p2 = c.C0 + xi2 * c.C1;
    const P poly = p0 + a * (p1 + a * (p2 + a * (P(1.0 / 6.0) + a * P(1.0 / 24.0))));
    return P(Lat<D, K>::w(d)) * c.rho * poly;
}

// Collision: f_out (post layout) from f (layout of a.f), the relaxation
// term R = omega (g - g^eq) and the per-sub-step Courant numbers nu_a =
// u_a / (r m), all in the population type.
template <typename P, int D, int K>
__global__ void __launch_bounds__(256) k_sub_collide(FieldArgs a, void *f_out, P *R, P *nu, double omega,
                                                     int m) {
    using L = Lat<D, K>;
    constexpr DirTable<D, K> dirs;
    const uint32_t x = blockIdx.x * 256u + threadIdx.x;
    if (x >= a.N) return;
    const int cx = x % a.n0, cy = (x / a.n0) % a.n1, cz = x / (a.n0 * a.n1);
    const int shift = a.layout == kLayoutStreamed ? 0 : 1;
    Mom M = {0.0, {0.0, 0.0, 0.0}, 0.0, 0.0};
    for (int i = 0; i < L::Q; ++i) {
        const int d = dirs.v[i];
        const double v = (double)fget<P, D, K>(a.f, a.blocked, a.N, src_slot<D, K>(a, i),
                                               src_index<D>(a, cx, cy, cz, d, shift));
        M.m0 += v;
        M.m1[0] += cx_of(d) * v;
        if (D >= 2) M.m1[1] += cy_of(d) * v;
        if (D >= 3) M.m1[2] += cz_of(d) * v;
        M.e2 += c2_of<D>(d) * v;
    }
    double gv[7];
    for (int j = 0; j < 7; ++j) {
        gv[j] = (double)pop<P>(a.g, j, a.N)[x];
        M.er += double((j - 3) * (j - 3)) * gv[j];
    }
    double rho, u[3] = {0.0, 0.0, 0.0}, T, Etot;
    finish_moments<D>(M, a.n_rot, rho, u, T, Etot);
    const FeqCoef<double> fc = feq_coef<double, D>(rho, u, T);
    for (int i = 0; i < L::Q; ++i) {
        const int d = dirs.v[i];
        const double v = (double)fget<P, D, K>(a.f, a.blocked, a.N, src_slot<D, K>(a, i),
                                               src_index<D>(a, cx, cy, cz, d, shift));
        reinterpret_cast<P *>(f_out)[pop_index(a.blocked, L::Q, a.N, i, x)] =
            (P)(v - omega * (v - feq_rt<double, D, K>(fc, d)));
    }
    const GeqCoef<double> gc = geq_coef<double>(T);
    static_for<0, 7>([&](auto J) {
        constexpr int j = decltype(J)::value;
        R[(size_t)j * a.N + x] = (P)(omega * (gv[j] - geq_dir<double, j>(gc)));
    });
    for (int d = 0; d < D; ++d) nu[(size_t)d * a.N + x] = (P)(u[d] / kR / m);
}

// One advection sub-step: dst = src - sum_a nu_a D_a[src] (- R on the last).
template <typename P, int D>
__global__ void __launch_bounds__(256) k_sub_advect(FieldArgs a, const P *src, P *dst, const P *nu,
                                                    const P *R) {
    const uint32_t x = blockIdx.x * 256u + threadIdx.x;
    if (x >= a.N) return;
    const int c[3] = {(int)(x % a.n0), (int)((x / a.n0) % a.n1), (int)(x / (a.n0 * a.n1))};
    const int n[3] = {a.n0, a.n1, a.n2}, op[3] = {a.open0, a.open1, a.open2};
    const uint32_t st[3] = {1u, (uint32_t)a.n0, (uint32_t)a.n0 * (uint32_t)a.n1};
    for (int j = 0; j < 7; ++j) {
        const P *h = src + (size_t)j * a.N;
        P adv = P(0);
        for (int ax = 0; ax < D; ++ax) {
            P v[5];
            for (int k = -2; k <= 2; ++k) {
                const int q = nb_coord(c[ax], k, n[ax], op[ax]);
                v[k + 2] = h[x + ((int64_t)q - c[ax]) * (int64_t)st[ax]];
            }
            adv += upwind3<P>(nu[(size_t)ax * a.N + x], v[0], v[1], v[2], v[3], v[4]);
        }
        P out = h[x] - adv;
        if (R) out -= R[(size_t)j * a.N + x];
        dst[(size_t)j * a.N + x] = out;
    }
}

template <typename P, int D, int K>
static hipError_t sub_step_t(const FieldArgs &a, void *f_out, void *g_out, void *scratch, int m, double omega,
                             hipStream_t s) {
    P *R = reinterpret_cast<P *>(scratch);
    P *nu = R + 7 * (size_t)a.N;
    P *gt = nu + 3 * (size_t)a.N;
    const dim3 g(blocks_for(a.N)), b(256);
    hipLaunchKernelGGL((k_sub_collide<P, D, K>), g, b, 0, s, a, f_out, R, nu, omega, m);
    const P *src = reinterpret_cast<const P *>(a.g);
    for (int k = 0; k < m; ++k) {
        P *dst = ((m - 1 - k) % 2 == 0) ? reinterpret_cast<P *>(g_out) : gt;
        hipLaunchKernelGGL((k_sub_advect<P, D>), g, b, 0, s, a, src, dst, nu, k == m - 1 ? R : (const P *)nullptr);
        src = dst;
    }
    return hipGetLastError();
}

hipError_t launch_step_sub(int dtype, int dim, int kind, const FieldArgs &a, void *f_out, void *g_out,
                           void *scratch, int m, double omega, hipStream_t s) {
    if (m < 2) return hipErrorInvalidValue;
    if (kind == kD2Q37) {
        if (dim != 2) return hipErrorInvalidValue;
        return dtype == 0 ? sub_step_t<float, 2, kD2Q37>(a, f_out, g_out, scratch, m, omega, s)
                          : sub_step_t<double, 2, kD2Q37>(a, f_out, g_out, scratch, m, omega, s);
    }
    if (dtype == 0) {
        if (dim == 1) return sub_step_t<float, 1, kTensor>(a, f_out, g_out, scratch, m, omega, s);
        if (dim == 2) return sub_step_t<float, 2, kTensor>(a, f_out, g_out, scratch, m, omega, s);
        return sub_step_t<float, 3, kTensor>(a, f_out, g_out, scratch, m, omega, s);
    }
    if (dim == 1) return sub_step_t<double, 1, kTensor>(a, f_out, g_out, scratch, m, omega, s);
    if (dim == 2) return sub_step_t<double, 2, kTensor>(a, f_out, g_out, scratch, m, omega, s);
    return sub_step_t<double, 3, kTensor>(a, f_out, g_out, scratch, m, omega, s);
}

// dst (blocked) <- src (plain); one thread per element of dst, read side
// gathered.
template <typename P>
__global__ void __launch_bounds__(256) k_to_blocked(int Q, uint32_t N, const P *src, P *dst) {
    const size_t e = (size_t)blockIdx.x * 256u + threadIdx.x;
    if (e >= (size_t)Q * N) return;
    const uint32_t lane = (uint32_t)(e % kBlk);
    const size_t bq = e / kBlk;
    const int i = (int)(bq % Q);
    const uint32_t x = (uint32_t)(bq / Q) * kBlk + lane;
    dst[e] = src[(size_t)i * N + x];
}

// Fixed-order sum of partials[nparts][K] (K <= 8).  series == NULL: the sums
// go to out[K].  Otherwise they are a row of the conservation series: row
// *slot of series[cap][K] receives them if *slot < cap, and *slot advances by
// one either way (the row counter lives in device memory, so a recorded
// sequence of steps does not depend on the absolute time it started at).
__global__ void __launch_bounds__(256) k_reduce(const double *partials, int nparts, int K,
                                                double *out, double *series, int64_t cap,
                                                int64_t *slot) {
    __shared__ double s[256];
    __shared__ double res[8];
    for (int k = 0; k < K; ++k) {
        double acc = 0.0;
        for (int p = threadIdx.x; p < nparts; p += 256) acc += partials[(size_t)p * K + k];
        s[threadIdx.x] = acc;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) res[k] = s[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *dst = out;
        if (series) {
            const int64_t row = *slot;
            dst = row >= 0 && row < cap ? series + row * K : nullptr;
            *slot = row + 1;
        }
        if (dst)
            for (int k = 0; k < K; ++k) dst[k] = res[k];
    }
}

// Quiet NaN into n values (debug poisoning of a step's destination).
template <typename P> __global__ void __launch_bounds__(256) k_fill_nan(P *p, size_t n) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = __builtin_nan("");
}

hipError_t launch_fill_nan(int dtype, void *p, size_t n, hipStream_t s) {
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    if (dtype == 0) hipLaunchKernelGGL(k_fill_nan<float>, g, b, 0, s, (float *)p, n);
    else hipLaunchKernelGGL(k_fill_nan<double>, g, b, 0, s, (double *)p, n);
    return hipGetLastError();
}

__global__ void k_set_i64(int64_t *p, int64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static unsigned blocks_for(uint32_t N) { return (N + 255u) / 256u; }

hipError_t launch_to_blocked(int dtype, int Q, uint32_t N, const void *src, void *dst, hipStream_t s) {
    if (N % kBlk) return hipErrorInvalidValue;
    const size_t n = (size_t)Q * N;
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    if (dtype == 0)
        hipLaunchKernelGGL(k_to_blocked<float>, g, b, 0, s, Q, N, (const float *)src, (float *)dst);
    else
        hipLaunchKernelGGL(k_to_blocked<double>, g, b, 0, s, Q, N, (const double *)src, (double *)dst);
    return hipGetLastError();
}

// Instantiate KERN<P, D, K> for the supported (dtype, dim, kind) and launch.
#define LBMX_DISPATCH_PDK(KERN, g, b, s, a)                                            \
    do {                                                                             \
        if (kind == kD2Q37) {                                                        \
            if (dim != 2) return hipErrorInvalidValue;                               \
            if (dtype == 0) hipLaunchKernelGGL((KERN<float, 2, kD2Q37>), g, b, 0, s, a); \
            else hipLaunchKernelGGL((KERN<double, 2, kD2Q37>), g, b, 0, s, a);       \
        } else if (dtype == 0) {                                                     \
            if (dim == 1) hipLaunchKernelGGL((KERN<float, 1, kTensor>), g, b, 0, s, a); \
            else if (dim == 2) hipLaunchKernelGGL((KERN<float, 2, kTensor>), g, b, 0, s, a); \
            else hipLaunchKernelGGL((KERN<float, 3, kTensor>), g, b, 0, s, a);        \
        } else {                                                                     \
            if (dim == 1) hipLaunchKernelGGL((KERN<double, 1, kTensor>), g, b, 0, s, a); \
            else if (dim == 2) hipLaunchKernelGGL((KERN<double, 2, kTensor>), g, b, 0, s, a); \
            else hipLaunchKernelGGL((KERN<double, 3, kTensor>), g, b, 0, s, a);       \
        }                                                                            \
    } while (0)

hipError_t launch_init(int dtype, int dim, int kind, const InitArgs &a, hipStream_t s) {
    const dim3 g(blocks_for(a.N)), b(256);
    LBMX_DISPATCH_PDK(k_init, g, b, s, a);
    return hipGetLastError();
}

int step_ntiles(int dim, const int tile[3], int n0, int n1, int n2, int *t0, int *t1, int *t2) {
    *t0 = (n0 + tile[0] - 1) / tile[0];
    *t1 = dim >= 2 ? (n1 + tile[1] - 1) / tile[1] : 1;
    *t2 = dim >= 3 ? n2 : 1;
    return *t0 * *t1 * *t2;
}

bool step_tile_supported(int dtype, int dim, int kind, const int tile[3]) {
    (void)dtype;
    bool ok = false;
#define C1(TXv, TYv) ok = ok || (dim == 1 && tile[0] == TXv && tile[1] == 1 && tile[2] == 1);
#define C2(TXv, TYv) ok = ok || (dim == 2 && tile[0] == TXv && tile[1] == TYv && tile[2] == 1);
#define C3(TXv, TYv) ok = ok || (dim == 3 && tile[0] == TXv && tile[1] == TYv && tile[2] == 1);
    if (kind == kD2Q37) {
        LBMX_TILES_37(C2)
        return ok;
    }
    LBMX_TILES_1D(C1)
    LBMX_TILES_2D(C2)
    LBMX_TILES_3D(C3)
#undef C1
#undef C2
#undef C3
    return ok;
}

hipError_t launch_step(int dtype, int dim, int kind, const int tile[3], const StepArgs &a, hipStream_t s) {
    if (kind == kD2Q37) return dtype == 0 ? launch_step_37_f32(tile, a, s) : launch_step_37_f64(tile, a, s);
    if (dim == 3) return launch_step_3(dtype, tile, a, s);
    return dtype == 0 ? launch_step_12_f32(dim, tile, a, s) : launch_step_12_f64(dim, tile, a, s);
}

hipError_t launch_fields(int dtype, int dim, int kind, const FieldArgs &a, int *nblocks, hipStream_t s) {
    const dim3 g(blocks_for(a.N)), b(256);
    *nblocks = (int)g.x;
    LBMX_DISPATCH_PDK(k_fields, g, b, s, a);
    return hipGetLastError();
}

hipError_t launch_export(int dtype, int dim, int kind, const FieldArgs &a, hipStream_t s) {
    const dim3 g(blocks_for(a.N)), b(256);
    LBMX_DISPATCH_PDK(k_export, g, b, s, a);
    return hipGetLastError();
}

hipError_t launch_reduce(const double *partials, int nparts, int K, double *out, hipStream_t s) {
    if (K < 1 || K > 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partials, nparts, K, out, (double *)nullptr,
                       (int64_t)0, (int64_t *)nullptr);
    return hipGetLastError();
}

hipError_t launch_reduce_series(const double *partials, int nparts, int K, double *series, int64_t cap,
                                int64_t *slot, hipStream_t s) {
    if (K < 1 || K > 8 || !series || !slot) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partials, nparts, K, (double *)nullptr, series,
                       cap, slot);
    return hipGetLastError();
}

hipError_t launch_set_i64(int64_t *p, int64_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

}  // namespace lbmx
