// Batched 1-D shock tubes (declared in include/lbm.h): many independent
// D1Q7 + D1Q7 tubes of uneven length, each with its own n, tau and number of
// steps, both ends open (zero-gradient clamp), advanced by ONE persistent
// launch.
//
// On-chip time loop: a tube of length L <= C (C = chunk capacity in nodes)
// is loaded into LDS once, advanced through all its steps there (one
// workgroup barrier per step) and written back.  A longer tube advances in
// passes of at most S steps: each pass covers the tube in chunks of C - 6S
// interior nodes plus 3S halo nodes per side (the update reaches 3 nodes per
// step), reads the pass's input buffer and writes the interior to the other
// buffer.  Every tube gets an even number of passes, so results end in f[0],
// g[0].
//
// Work distribution, in two phases of the same launch:
//  1. long tubes, pass by pass, through a device work queue of chunks: the
//     chunks of pass 0 of every long tube start in the queue; the workgroup
//     that completes the last chunk of a tube's pass enqueues the chunks of
//     its next pass (or finishes the tube: last pass, or a failure).  Any
//     workgroup takes any queued chunk, so a long tube runs on as many
//     compute units as it has chunks, no chunk ever waits for another, and a
//     failed tube stops producing work.
//  2. tubes that fit on chip, longest work first (a one-workgroup bitonic
//     sort orders them), popped from a device counter -- by workgroups that
//     find the chunk queue empty (all but a few reserved ones) and by every
//     workgroup once the long tubes are done.
//
// Per node and step the arithmetic is that of the per-step kernels (Sec. V
// B): FP64 moments and temperature, fourth-order Hermite equilibria, BGK
// with the conservative FP32 correction, third-order upwind advection of the
// rotational populations.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <mutex>
#include <string>
#include <vector>

#include "launch.hpp"
#include "lbm.h"
#include "lbm_device.hpp"

namespace lbmx {

struct BatchArgs {
    const int64_t *offsets;
    const double *n_rot, *tau;
    const int64_t *nsteps;
    void *f[2], *g[2];  // packed [7][total]
    int32_t *status;
    int64_t *steps_done;  // may be NULL
    int32_t *order;     // workspace: on-chip tubes in processing order (nwhole of them)
    int32_t *counter;   // workspace: see kCtr*
    int32_t *ltube;     // workspace: long tubes, most passes first (nlong)
    int32_t *lpas;      // workspace: their pass counts (non-increasing)
    int32_t *lpfx;      // workspace: prefix sums of their chunk counts (nlong + 1)
    int32_t *pdone;     // workspace: chunks completed per long tube, all passes (nlong)
    int32_t *tpass;     // workspace: pass whose chunks a long tube has queued (nlong)
    int64_t *qitem;     // workspace: chunk queue slots, (long-tube index << 32) | chunk
    int64_t *qseq;      // workspace: slot sequence: 2 pos + 1 = item of position pos
                        //            ready; 2 pos = free for position pos
    int qcap;           // slots in the queue (twice the chunks of one pass of all long tubes)
    int64_t *fail_at;   // workspace: first failure of a long tube, fail_key (INT64_MAX: none)
    int num;
    uint32_t total;
    int chunk;      // nodes per LDS buffer
    int superstep;  // steps per pass of a chunked tube
    int m;          // rotational advection sub-steps per step (1: the update as written)
    int hw;         // halo nodes a step reaches: max(3, 2 m)
};

// counter[]: on-chip tube queue head, chunk queue head and tail, on-chip and
// long tube counts, long tubes not yet finished.
constexpr int kCtrQueue = 0, kCtrHead = 1, kCtrTail = 2, kCtrWhole = 3, kCtrLong = 4, kCtrRemain = 5;
constexpr int kCtrWords = 64, kMaxGrid = 1024;
constexpr int64_t kNoFail = 0x7fffffffffffffffLL;
// Failure record of a long tube: the smallest key over its chunks wins, i.e.
// the earliest failing step and, at that step, the most severe kind -- what
// the whole tube on chip would report.
__device__ __forceinline__ int64_t fail_key(int64_t step, int kind) { return (step << 8) | (255 - kind); }
// Status of a long tube that did not finish (a bounded wait of the chunk
// queue gave up; never expected).
constexpr int32_t kStatusAborted = 4;
// Workgroups that keep polling the chunk queue instead of taking on-chip
// tubes while long tubes run (the long tubes' passes are the critical path).
constexpr int kReserve = 16;
// Largest number of chunk passes (passes x chunks over all long tubes) of one
// launch: queue positions and completion counts are int32.
constexpr int64_t kMaxTickets = 1LL << 30;

// Passes of a chunked tube: at most S steps each, at least 2, even.
__host__ __device__ inline int64_t tube_passes(int64_t steps, int S) {
    int64_t p = (steps + S - 1) / S;
    if (p < 2) p = 2;
    if (p & 1) ++p;
    return p;
}

// ---------------------------------------------------------------------------
// Schedule (one workgroup): resets the queue counters; on-chip tubes sorted
// by work (length x steps, descending) into order[0..nwhole); long tubes
// (L > C) sorted by step count (descending) into ltube[0..nlong) with their
// pass counts and the prefix sums of their chunk counts, and the chunks of
// their pass 0 placed in the chunk queue.  Bitonic sorts of 64-bit keys (value << 24 | 2^24 - 1 - index) in
// LDS.  Batches of more than kSortMax tubes, or whose long tubes would need
// more than kMaxTickets chunk passes, keep index order and run every tube in
// phase 2 (a long tube then walks its chunks on one workgroup).
// ---------------------------------------------------------------------------
constexpr int kSortMax = 16384;

__device__ void bitonic_desc(unsigned long long *key, int P2) {
    for (int size = 2; size <= P2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P2; i += 1024) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool desc = (i & size) == 0;
                    const unsigned long long ki = key[i], kj = key[j];
                    if (desc ? (ki < kj) : (ki > kj)) {
                        key[i] = kj;
                        key[j] = ki;
                    }
                }
            }
            __syncthreads();
        }
    }
}

__global__ void __launch_bounds__(1024) k_batch_order(BatchArgs a) {
    __shared__ unsigned long long key[kSortMax];
    __shared__ int s_cnt[2];
    __shared__ int part[1024];
    const int n = a.num;
    const int inner = a.chunk - 2 * a.hw * a.superstep;
    if (threadIdx.x == 0) {
        a.counter[kCtrQueue] = 0;
        a.counter[kCtrHead] = 0;
        a.counter[kCtrTail] = 0;
        a.counter[kCtrRemain] = 0;
        s_cnt[0] = 0;
        s_cnt[1] = 0;
    }
    for (int i = threadIdx.x; i < n; i += 1024) a.fail_at[i] = kNoFail;
    if (n > kSortMax) {
        for (int i = threadIdx.x; i < n; i += 1024) a.order[i] = i;
        if (threadIdx.x == 0) {
            a.counter[kCtrWhole] = n;
            a.counter[kCtrLong] = 0;
            a.lpfx[0] = 0;
        }
        return;
    }
    // Tubes with no steps to run are finished here, as the queues would
    // finish them: populations left in f[0] / g[0], no step taken, status 0
    // (3 for an empty tube).  A call that advances a few tubes of a large
    // batch then costs only those tubes' work.
    for (int i = threadIdx.x; i < n; i += 1024)
        if (a.nsteps[i] <= 0) {
            a.status[i] = a.offsets[i + 1] > a.offsets[i] ? 0 : 3;
            if (a.steps_done) a.steps_done[i] = 0;
        }
    int P2 = 1;
    while (P2 < n) P2 <<= 1;
    __syncthreads();
    // 1. on-chip tubes by work
    for (int i = threadIdx.x; i < P2; i += 1024) {
        unsigned long long k = 0;
        if (i < n) {
            const long long L = a.offsets[i + 1] - a.offsets[i];
            if (L <= a.chunk && a.nsteps[i] > 0) {
                long long w = L * a.nsteps[i];
                if (w > (1LL << 39) - 1) w = (1LL << 39) - 1;
                k = ((unsigned long long)w << 24) | (unsigned long long)((1 << 24) - 1 - i);
                atomicAdd(&s_cnt[0], 1);
            }
        }
        key[i] = k;
    }
    __syncthreads();
    bitonic_desc(key, P2);
    const int nw = s_cnt[0];
    for (int i = threadIdx.x; i < nw; i += 1024) a.order[i] = (1 << 24) - 1 - (int)(key[i] & ((1ULL << 24) - 1));
    __syncthreads();
    // 2. long tubes by steps
    for (int i = threadIdx.x; i < P2; i += 1024) {
        unsigned long long k = 0;
        if (i < n) {
            const long long L = a.offsets[i + 1] - a.offsets[i];
            if (L > a.chunk && a.nsteps[i] > 0) {
                long long st = a.nsteps[i];
                if (st > (1LL << 39) - 2) st = (1LL << 39) - 2;
                k = ((unsigned long long)(st + 1) << 24) | (unsigned long long)((1 << 24) - 1 - i);
                atomicAdd(&s_cnt[1], 1);
            }
        }
        key[i] = k;
    }
    __syncthreads();
    bitonic_desc(key, P2);
    const int nl = s_cnt[1];
    // chunk counts -> segment sums per thread -> prefix
    const int seg = (nl + 1023) / 1024;
    int sum = 0;
    for (int j = threadIdx.x * seg; j < nl && j < (threadIdx.x + 1) * seg; ++j) {
        const int t = (1 << 24) - 1 - (int)(key[j] & ((1ULL << 24) - 1));
        const int64_t L = a.offsets[t + 1] - a.offsets[t];
        const int64_t st = a.nsteps[t] > 0 ? a.nsteps[t] : 0;
        a.ltube[j] = t;
        a.lpas[j] = (int)tube_passes(st, a.superstep);
        sum += (int)((L + inner - 1) / inner);
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int w = 0; w < 1024; ++w) {
            const int v = part[w];
            part[w] = acc;
            acc += v;
        }
        a.lpfx[nl] = acc;
        a.counter[kCtrWhole] = nw;
        a.counter[kCtrLong] = nl;
    }
    __syncthreads();
    int acc = part[threadIdx.x];
    for (int j = threadIdx.x * seg; j < nl && j < (threadIdx.x + 1) * seg; ++j) {
        a.lpfx[j] = acc;
        a.pdone[j] = 0;
        a.tpass[j] = 0;
        const int t = a.ltube[j];
        const int64_t L = a.offsets[t + 1] - a.offsets[t];
        acc += (int)((L + inner - 1) / inner);
        a.status[t] = kStatusAborted;  // until the tube finishes
        if (a.steps_done) a.steps_done[t] = 0;
    }
    // chunk passes of phase 1 (passes x chunks of every long tube)
    __shared__ unsigned long long s_tk;
    if (threadIdx.x == 0) s_tk = 0;
    __syncthreads();
    unsigned long long tk = 0;
    for (int j = threadIdx.x * seg; j < nl && j < (threadIdx.x + 1) * seg; ++j) {
        const int t = a.ltube[j];
        const int64_t L = a.offsets[t + 1] - a.offsets[t];
        const int64_t st = a.nsteps[t] > 0 ? a.nsteps[t] : 0;
        tk += (unsigned long long)tube_passes(st, a.superstep) * (unsigned long long)((L + inner - 1) / inner);
    }
    atomicAdd(&s_tk, tk);
    __syncthreads();
    if (s_tk >= (unsigned long long)kMaxTickets) {  // too many: everything in phase 2, index order
        for (int i = threadIdx.x; i < n; i += 1024) a.order[i] = i;
        if (threadIdx.x == 0) {
            a.counter[kCtrWhole] = n;
            a.counter[kCtrLong] = 0;
        }
        return;
    }
    // chunk queue: the chunks of pass 0 of every long tube at positions
    // [0, lpfx[nl]), in long-tube order; every other slot free
    const int np0 = a.lpfx[nl];
    for (int q = threadIdx.x; q < a.qcap; q += 1024) a.qseq[q] = 2 * (int64_t)q;
    __syncthreads();
    for (int j = threadIdx.x * seg; j < nl && j < (threadIdx.x + 1) * seg; ++j)
        for (int q = a.lpfx[j]; q < a.lpfx[j + 1]; ++q) {
            a.qitem[q] = ((int64_t)j << 32) | (int64_t)(q - a.lpfx[j]);
            a.qseq[q] = 2 * (int64_t)q + 1;
        }
    if (threadIdx.x == 0) {
        a.counter[kCtrTail] = np0;
        a.counter[kCtrRemain] = nl;
    }
}

// ---------------------------------------------------------------------------
// One node's update from LDS (region of R nodes, local clamp at the region
// edges).  F, G: [7][C] arrays; shift = 0 if F holds streamed populations,
// 1 if post-collision ones (gathered from x - c).
// ---------------------------------------------------------------------------
// ADV = false (sub-stepped rotational advection): go receives the
// relaxation increment rl instead of g - adv + rl, *nu_out the Courant number.
template <typename P, bool ADV = true>
__device__ __forceinline__ void lds_node(const P *F, const P *G, int C, int x, int R, int shift,
                                         P om, double omega, double n_rot, P (&fo)[7], P (&go)[7],
                                         double &rho, double &T, P *nu_out = nullptr) {
    P fv[7], gv[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        int s = x - (i - 3) * shift;
        s = s < 0 ? 0 : (s >= R ? R - 1 : s);
        fv[i] = F[i * C + s];
    }
#pragma unroll
    for (int j = 0; j < 7; ++j) gv[j] = G[j * C + x];
    Mom M = {0.0, {0.0, 0.0, 0.0}, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const double v = (double)fv[i], c = i - 3;
        M.m0 += v;
        M.m1[0] += c * v;
        M.e2 += c * c * v;
    }
#pragma unroll
    for (int j = 0; j < 7; ++j)
        if (j != 3) M.er += double((j - 3) * (j - 3)) * (double)gv[j];
    double u[3] = {0.0, 0.0, 0.0}, Etot;
    const double inv = finish_moments<1>(M, n_rot, rho, u, T, Etot);

    const P up[3] = {(P)u[0], P(0), P(0)};
    const FeqCoef<P> fc = feq_coef<P, 1>((P)rho, up, (P)T);
    P d[7];
    static_for<0, 3>([&](auto I) {
        constexpr int i = decltype(I)::value;
        P fp, fm;
        feq_pair<P, 1, i>(fc, fp, fm);
        d[i] = om * (fp - fv[i]);
        d[6 - i] = om * (fm - fv[6 - i]);
    });
    d[3] = om * (P(w_of<1>(3)) * fc.rho * fc.A0 - fv[3]);
    if constexpr (sizeof(P) == 4) {
        // conservative FP32 relaxation: defects to the rest and +-1 populations
        P s0 = P(0), s1 = P(0), s2 = P(0);
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            const P c = P(i - 3);
            s0 += d[i];
            s1 += c * d[i];
            s2 += c * c * d[i];
        }
        const double t2 = omega * (M.m1[0] * M.m1[0] * inv + rho * T * kInvR2 - M.e2);
        const double R1[3] = {-(double)s1, 0.0, 0.0};
        const Eps ep = eps_from_defects<1>(-(double)s0, R1, t2 - (double)s2);
        d[3] += (P)ep.e[0];
        d[2] += (P)ep.e[1];
        d[4] += (P)ep.e[2];
    }
#pragma unroll
    for (int i = 0; i < 7; ++i) fo[i] = fv[i] + d[i];

    const GeqCoef<P> gc = geq_coef<P>((P)T);
    const P nu = up[0] * P(1.0 / kR);
    const int xm2 = x - 2 < 0 ? 0 : x - 2, xm1 = x - 1 < 0 ? 0 : x - 1;
    const int xp1 = x + 1 >= R ? R - 1 : x + 1, xp2 = x + 2 >= R ? R - 1 : x + 2;
    P adv[7], rl[7];
    static_for<0, 7>([&](auto J) {
        constexpr int j = decltype(J)::value;
        if constexpr (ADV)
            adv[j] = upwind3<P>(nu, G[j * C + xm2], G[j * C + xm1], gv[j], G[j * C + xp1], G[j * C + xp2]);
        rl[j] = om * (geq_dir<P, j>(gc) - gv[j]);
    });
    if constexpr (sizeof(P) == 4) {
        double r0 = 0.0, r2 = 0.0, g0 = 0.0;
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            r0 += (double)rl[j];
            r2 += double((j - 3) * (j - 3)) * (double)rl[j];
            g0 += (double)gv[j];
        }
        double al, ga;
        gfix_from_defects(omega * (1.0 - g0) - r0, omega * (T * kInvR2 - M.er) - r2, al, ga);
#pragma unroll
        for (int j = 0; j < 7; ++j)
            rl[j] += P(kW1[iabs(j - 3)]) * ((P)al + P((j - 3) * (j - 3)) * (P)ga);
    }
    if constexpr (ADV) {
#pragma unroll
        for (int j = 0; j < 7; ++j) go[j] = gv[j] - adv[j] + rl[j];
    } else {
#pragma unroll
        for (int j = 0; j < 7; ++j) go[j] = rl[j];
        *nu_out = nu;
    }
}

// 0 healthy, 1 non-finite, 2 rho <= 0 or T <= 0.
__device__ __forceinline__ int health(double rho, double T) {
    if (!__builtin_isfinite(rho) || !__builtin_isfinite(T)) return 1;
    return (rho <= 0.0 || T <= 0.0) ? 2 : 0;
}

// Advance the region [0, R) held in LDS buffer `cur` by `steps` steps,
// ping-ponging between the two LDS buffers (one barrier per step).  `shift`
// is the representation in `cur` on entry (0 streamed, 1 post-collision).
// Nodes [vlo, vhi) are health-checked each step (their values are exact at
// every step); on failure the loop stops.  bad[2] (LDS, zero on entry)
// receives the failure kind in slot (step & 1): a thread can write slot
// (s & 1) again only at step s + 2, after every thread has passed the
// barrier of step s + 1 and so has read the flag of step s -- all threads
// leave at the same step.  Returns the buffer index holding the result;
// *shift_out its representation.
// The rotational advection in m > 1 sub-steps (BatchArgs::m): per step, the
// collision of every node (f to the other buffer, the rotational relaxation
// increment and Courant number kept in registers, NPT nodes per thread),
// then m advection passes over G with Courant number nu / m, one barrier
// each, the last adding the relaxation increment.  g(t+1) = A^m g(t) + rl.
// The translational and rotational buffers then alternate independently:
// *gcur_out receives the index of the buffer holding g.
template <typename P, int B>
__device__ int lds_run_sub(P *F, P *G, int C, int R, int steps, int shift, P om, double omega,
                           double n_rot, int m, int vlo, int vhi, int *bad, int *shift_out, int *ran,
                           int *gcur_out) {
    constexpr int NPT = (1536 + B - 1) / B;  // nodes per thread: C <= 1536
    int cur = 0, gc = 0;
    *ran = 0;
    const P minv = P(1) / P(m);
    for (int s = 0; s < steps; ++s) {
        const P *Fi = F + cur * 7 * C;
        P *Fo = F + (cur ^ 1) * 7 * C;
        P rl[NPT][7], nu[NPT];
        int h = 0;
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int x = (int)threadIdx.x + k * B;
            if (x < R) {
                P fo[7];
                double rho, T;
                lds_node<P, false>(Fi, G + gc * 7 * C, C, x, R, shift, om, omega, n_rot, fo, rl[k], rho, T, &nu[k]);
                nu[k] *= minv;
#pragma unroll
                for (int i = 0; i < 7; ++i) Fo[i * C + x] = fo[i];
                if (x >= vlo && x < vhi) {
                    const int hh = health(rho, T);
                    h = hh > h ? hh : h;
                }
            }
        }
        for (int q = 0; q < m; ++q) {
            const P *Gs = G + (gc ^ (q & 1)) * 7 * C;
            P *Gd = G + (gc ^ ((q & 1) ^ 1)) * 7 * C;
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int x = (int)threadIdx.x + k * B;
                if (x < R) {
                    const int xm2 = x - 2 < 0 ? 0 : x - 2, xm1 = x - 1 < 0 ? 0 : x - 1;
                    const int xp1 = x + 1 >= R ? R - 1 : x + 1, xp2 = x + 2 >= R ? R - 1 : x + 2;
#pragma unroll
                    for (int j = 0; j < 7; ++j) {
                        const P *gj = Gs + j * C;
                        P v = gj[x] - upwind3<P>(nu[k], gj[xm2], gj[xm1], gj[x], gj[xp1], gj[xp2]);
                        if (q == m - 1) v += rl[k][j];
                        Gd[j * C + x] = v;
                    }
                }
            }
            __syncthreads();
        }
        if (h) atomicMax(&bad[s & 1], h);
        shift = 1;
        cur ^= 1;
        gc ^= m & 1;
        *ran = s + 1;
        __syncthreads();
        if (bad[s & 1]) break;
    }
    *shift_out = shift;
    *gcur_out = gc;
    return cur;
}

// SUB: the kernel variant for m > 1 (a separate instantiation, so that the
// register allocation of the update as written does not change).
template <typename P, int B, bool SUB>
__device__ int lds_run(P *F, P *G, int C, int R, int steps, int shift, P om, double omega,
                       double n_rot, int m, int vlo, int vhi, int *bad, int *shift_out, int *ran, int *gcur_out) {
    if constexpr (SUB)
        return lds_run_sub<P, B>(F, G, C, R, steps, shift, om, omega, n_rot, m, vlo, vhi, bad, shift_out, ran,
                                 gcur_out);
    int cur = 0;
    *ran = 0;
    for (int s = 0; s < steps; ++s) {
        const P *Fi = F + cur * 7 * C, *Gi = G + cur * 7 * C;
        P *Fo = F + (cur ^ 1) * 7 * C, *Go = G + (cur ^ 1) * 7 * C;
        int h = 0;
#pragma unroll 1
        for (int x = threadIdx.x; x < R; x += B) {
            P fo[7], go[7];
            double rho, T;
            lds_node<P>(Fi, Gi, C, x, R, shift, om, omega, n_rot, fo, go, rho, T);
#pragma unroll
            for (int i = 0; i < 7; ++i) Fo[i * C + x] = fo[i];
#pragma unroll
            for (int j = 0; j < 7; ++j) Go[j * C + x] = go[j];
            if (x >= vlo && x < vhi) {
                const int hh = health(rho, T);
                h = hh > h ? hh : h;
            }
        }
        if (h) atomicMax(&bad[s & 1], h);
        shift = 1;
        cur ^= 1;
        *ran = s + 1;
        __syncthreads();
        if (bad[s & 1]) break;
    }
    *shift_out = shift;
    *gcur_out = cur;
    return cur;
}

// Bounded polls of the chunk queue (a sleep each): an idle workgroup gives up
// after ~5-15 s without work (the others go on), a pusher's wait for a free
// slot after ~1e6 polls (never expected: the slot's consumer is a running
// workgroup).
constexpr long kIdleSpins = 1L << 22, kSlotSpins = 1L << 20;

__device__ __forceinline__ bool wait_seq(const int64_t *seq, int64_t want) {
    long spins = 0;
    while (__hip_atomic_load(seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != want) {
        if (++spins > kSlotSpins) return false;
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

// Thread 0: the next piece of work.  1: a queued chunk (*x = long-tube
// index, *y = chunk); 2: an on-chip tube (*x = its queue position); 0: the
// long tubes are done (or this workgroup gave up waiting).  Chunk positions
// are claimed by fetch-and-add once the queue looks non-empty; a claim that
// lost the race waits for a later push to fill its position, or for the end
// of the long tubes (then nothing will fill it).
__device__ int next_work(const BatchArgs &a, int nwhole, bool &p2_open, int *x, int *y) {
    int32_t *ctr = a.counter;
    long spins = 0;
    for (;;) {
        const int h = __hip_atomic_load(&ctr[kCtrHead], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int tl = __hip_atomic_load(&ctr[kCtrTail], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (h < tl) {
            const int q = atomicAdd(&ctr[kCtrHead], 1);
            const int slot = q % a.qcap;
            const int64_t want = 2 * (int64_t)q + 1;
            for (long w = 0;; ++w) {
                if (__hip_atomic_load(&a.qseq[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == want) break;
                if (__hip_atomic_load(&ctr[kCtrRemain], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <= 0 ||
                    w > kIdleSpins)
                    return 0;
                __builtin_amdgcn_s_sleep(1);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const int64_t it = a.qitem[slot];
            __hip_atomic_store(&a.qseq[slot], 2 * ((int64_t)q + a.qcap), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
            *x = (int)(it >> 32);
            *y = (int)(it & 0xffffffff);
            return 1;
        }
        if (__hip_atomic_load(&ctr[kCtrRemain], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <= 0) return 0;
        if (p2_open && (int)blockIdx.x >= kReserve) {
            const int it = atomicAdd(&ctr[kCtrQueue], 1);
            if (it < nwhole) {
                *x = it;
                return 2;
            }
            p2_open = false;
        }
        if (++spins > kIdleSpins) return 0;
        __builtin_amdgcn_s_sleep(4);
    }
}

// LDS <- rows [0, 7) x nodes [0, R) of f and g starting at packed node
// `first`; four elements per thread and iteration, all loads issued before
// the LDS stores, so that several global loads are in flight.
template <typename P, int B>
__device__ __forceinline__ void load_region(P *F, P *G, int C, const P *fs, const P *gs, uint32_t tot,
                                            int64_t first, int R) {
    const int n = 7 * R;
    for (int e0 = threadIdx.x; e0 < n; e0 += 4 * B) {
        P fv[4], gv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * B;
            if (e < n) {
                const int i = e / R, x = e - i * R;
                fv[u] = fs[(size_t)i * tot + first + x];
                gv[u] = gs[(size_t)i * tot + first + x];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * B;
            if (e < n) {
                const int i = e / R, x = e - i * R;
                F[i * C + x] = fv[u];
                G[i * C + x] = gv[u];
            }
        }
    }
    __syncthreads();
}

// One chunk of one pass of a long tube: nodes [c0, c1) with a halo of 3 sp
// nodes per side read from (fs, gs), advanced sp steps in LDS, the interior
// written to (fd, gd).  Returns the steps completed (sp unless a node of the
// interior failed the health check, *bad then holds its kind).
template <typename P, int B, bool SUB>
__device__ int run_chunk(P *F, P *G, int C, const P *fs, const P *gs, P *fd, P *gd, uint32_t tot, int64_t base,
                         int L, int c0, int c1, int sp, P om, double omega, double n_rot, int m, int hw,
                         int *bad) {
    const int halo = hw * sp;
    const int lo = c0 - halo > 0 ? c0 - halo : 0;
    const int hi = c1 + halo < L ? c1 + halo : L;
    const int R = hi - lo;
    load_region<P, B>(F, G, C, fs, gs, tot, base + lo, R);
    int shift, ran, gcur;
    const int cur = lds_run<P, B, SUB>(F, G, C, R, sp, 0, om, omega, n_rot, m, c0 - lo, c1 - lo, bad, &shift,
                                       &ran, &gcur);
    const P *Fr = F + cur * 7 * C, *Gr = G + gcur * 7 * C;
    const int W = c1 - c0;
    for (int e = threadIdx.x; e < 7 * W; e += B) {
        const int i = e / W, x = (c0 - lo) + (e - i * W);
        int sx = x - (i - 3) * shift;
        sx = sx < 0 ? 0 : (sx >= R ? R - 1 : sx);
        fd[(size_t)i * tot + base + lo + x] = Fr[i * C + sx];
        gd[(size_t)i * tot + base + lo + x] = Gr[i * C + x];
    }
    __syncthreads();
    return ran;
}

// One tube of the on-chip queue (queue position `item`): its whole time loop
// on chip, or, in index-order mode, its passes chunk by chunk on this
// workgroup.  Writes its status and steps.  s_bad: LDS flags, zero on entry.
template <typename P, int B, bool SUB>
__device__ void whole_tube(const BatchArgs &a, int item, P *F, P *G, int C, int *s_bad) {
    const uint32_t tot = a.total;
    const int t = a.order[item];
    const int64_t base = a.offsets[t];
    const int L = (int)(a.offsets[t + 1] - base);
    if (L < 1) {  // empty tube: nothing to advance
        if (threadIdx.x == 0) {
            a.status[t] = 3;
            if (a.steps_done) a.steps_done[t] = 0;
        }
        __syncthreads();
        return;
    }
    const int64_t steps = a.nsteps[t] > 0 ? a.nsteps[t] : 0;
    const double omega = 1.0 / a.tau[t], n_rot = a.n_rot[t];
    const P om = (P)omega;
    int64_t done_total = 0;
    const P *f0 = reinterpret_cast<const P *>(a.f[0]);
    const P *g0 = reinterpret_cast<const P *>(a.g[0]);

    if (L <= C) {
        // whole tube on chip
        load_region<P, B>(F, G, C, f0, g0, tot, base, L);
        int shift, ran, gcur;
        const int cur = lds_run<P, B, SUB>(F, G, C, L, (int)steps, 0, om, omega, n_rot, a.m, 0, L, s_bad, &shift,
                                           &ran, &gcur);
        done_total = ran;
        const P *Fr = F + cur * 7 * C, *Gr = G + gcur * 7 * C;
        P *f0w = reinterpret_cast<P *>(a.f[0]);
        P *g0w = reinterpret_cast<P *>(a.g[0]);
        // back to streamed form: f(x) = f*(clamp(x - c))
        for (int e = threadIdx.x; e < 7 * L; e += B) {
            const int i = e / L, x = e - i * L;
            int sx = x - (i - 3) * shift;
            sx = sx < 0 ? 0 : (sx >= L ? L - 1 : sx);
            f0w[(size_t)i * tot + base + x] = Fr[i * C + sx];
            g0w[(size_t)i * tot + base + x] = Gr[i * C + x];
        }
    } else {
        // passes of `superstep` steps over halo'd chunks; even pass count
        const int S0 = a.superstep;
        int passes = (int)((steps + S0 - 1) / S0);
        if (passes < 2) passes = 2;
        if (passes & 1) ++passes;
        int64_t done = 0;
        for (int p = 0; p < passes && !(s_bad[0] | s_bad[1]); ++p) {
            const int sp = (int)((steps - done) / (passes - p));
            const P *fs = reinterpret_cast<const P *>(a.f[p & 1]);
            const P *gs = reinterpret_cast<const P *>(a.g[p & 1]);
            P *fd = reinterpret_cast<P *>(a.f[(p + 1) & 1]);
            P *gd = reinterpret_cast<P *>(a.g[(p + 1) & 1]);
            const int halo = a.hw * sp;
            const int inner = C - 2 * halo;  // > 0 by the host's choice of superstep
            int pass_ran = sp;
            for (int c0 = 0; c0 < L; c0 += inner) {
                const int c1 = c0 + inner < L ? c0 + inner : L;
                const int lo = c0 - halo > 0 ? c0 - halo : 0;
                const int hi = c1 + halo < L ? c1 + halo : L;
                const int R = hi - lo;
                load_region<P, B>(F, G, C, fs, gs, tot, base + lo, R);
                int shift, ran, gcur;
                const int cur = lds_run<P, B, SUB>(F, G, C, R, sp, 0, om, omega, n_rot, a.m, c0 - lo, c1 - lo,
                                                   s_bad, &shift, &ran, &gcur);
                pass_ran = ran < pass_ran ? ran : pass_ran;
                const P *Fr = F + cur * 7 * C, *Gr = G + gcur * 7 * C;
                const int W = c1 - c0;
                for (int e = threadIdx.x; e < 7 * W; e += B) {
                    const int i = e / W, x = (c0 - lo) + (e - i * W);
                    int sx = x - (i - 3) * shift;
                    sx = sx < 0 ? 0 : (sx >= R ? R - 1 : sx);
                    fd[(size_t)i * tot + base + lo + x] = Fr[i * C + sx];
                    gd[(size_t)i * tot + base + lo + x] = Gr[i * C + x];
                }
                __syncthreads();
            }
            done_total = done + pass_ran;
            done += sp;
            __threadfence();
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        a.status[t] = s_bad[0] > s_bad[1] ? s_bad[0] : s_bad[1];
        if (a.steps_done) a.steps_done[t] = done_total;
    }
    __syncthreads();
}

template <typename P, int B, bool SUB>
__global__ void __launch_bounds__(B) k_batch(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int C = a.chunk;
    P *F = reinterpret_cast<P *>(smem_raw);  // [2][7][C]
    P *G = F + 14 * C;                        // [2][7][C]
    __shared__ int s_item, s_bad[2];
    const uint32_t tot = a.total;
    const int nwhole = a.counter[kCtrWhole];

    // Phase 1: chunks of the long tubes from the queue; on-chip tubes while
    // the queue is empty.  Phase 2: the remaining on-chip tubes.
    const int nlong = a.counter[kCtrLong];
    const int inner = C - 2 * a.hw * a.superstep;
    __shared__ int s_kind, s_x, s_y, s_last, s_pos;
    bool p2_open = true;  // thread 0's view of the on-chip queue
    while (nlong > 0) {
        if (threadIdx.x == 0) {
            int x = 0, y = 0;
            s_kind = next_work(a, nwhole, p2_open, &x, &y);
            s_x = x;
            s_y = y;
            s_bad[0] = s_bad[1] = 0;
        }
        __syncthreads();
        const int kind = s_kind, jl = s_x, k = s_y;
        __syncthreads();
        if (kind == 0) break;  // uniform
        if (kind == 2) {
            whole_tube<P, B, SUB>(a, jl, F, G, C, s_bad);
            continue;
        }
        // chunk k of the queued pass of long tube jl
        const int t = a.ltube[jl];
        const int nch = a.lpfx[jl + 1] - a.lpfx[jl];
        const int p = __hip_atomic_load(&a.tpass[jl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int64_t steps = a.nsteps[t] > 0 ? a.nsteps[t] : 0;
        const int64_t passes = a.lpas[jl];
        const int64_t done = steps * p / passes;
        if (threadIdx.x == 0) {  // failed in an earlier pass?  (A failure in this pass still lets
                                 // every chunk of the pass run: the earliest step must be found.)
            const int64_t f = __hip_atomic_load(&a.fail_at[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_item = f != kNoFail && (f >> 8) <= done;
        }
        __syncthreads();
        if (!s_item) {
            const int sp = (int)(steps * (p + 1) / passes - done);
            const int c0 = k * inner;
            const int L = (int)(a.offsets[t + 1] - a.offsets[t]);
            const int c1 = c0 + inner < L ? c0 + inner : L;
            const double omega = 1.0 / a.tau[t], n_rot = a.n_rot[t];
            const int ran = run_chunk<P, B, SUB>(F, G, C, reinterpret_cast<const P *>(a.f[p & 1]),
                                            reinterpret_cast<const P *>(a.g[p & 1]),
                                            reinterpret_cast<P *>(a.f[(p + 1) & 1]),
                                            reinterpret_cast<P *>(a.g[(p + 1) & 1]), tot, a.offsets[t], L, c0,
                                            c1, sp, (P)omega, omega, n_rot, a.m, a.hw, s_bad);
            const int fail = s_bad[0] > s_bad[1] ? s_bad[0] : s_bad[1];
            if (threadIdx.x == 0 && fail)
                __hip_atomic_fetch_min(&a.fail_at[t], fail_key(done + ran, fail), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();  // every wave's stores have reached the cache
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const int old = __hip_atomic_fetch_add(&a.pdone[jl], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int last = 0;
            if (old + 1 == (p + 1) * nch) {  // the pass is complete: finish the tube or queue the next pass
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                const int64_t f = __hip_atomic_load(&a.fail_at[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (f != kNoFail || p + 1 >= passes) {
                    a.status[t] = f != kNoFail ? 255 - (int)(f & 255) : 0;
                    if (a.steps_done) a.steps_done[t] = f != kNoFail ? f >> 8 : steps;
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    __hip_atomic_fetch_add(&a.counter[kCtrRemain], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    __hip_atomic_store(&a.tpass[jl], p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    s_pos = atomicAdd(&a.counter[kCtrTail], nch);
                    last = 1;
                }
            }
            s_last = last;
        }
        __syncthreads();
        if (s_last) {  // publish the next pass's chunks
            for (int c = threadIdx.x; c < nch; c += B) {
                const int q = s_pos + c, slot = q % a.qcap;
                if (!wait_seq(&a.qseq[slot], 2 * (int64_t)q)) continue;  // lost: the tube stays unfinished
                a.qitem[slot] = ((int64_t)jl << 32) | (int64_t)c;
                __hip_atomic_store(&a.qseq[slot], 2 * (int64_t)q + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
    }

    // Phase 2: the on-chip tubes still queued (every tube when the schedule
    // kept index order).
    for (;;) {
        if (threadIdx.x == 0) {
            s_item = atomicAdd(&a.counter[kCtrQueue], 1);
            s_bad[0] = s_bad[1] = 0;
        }
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= nwhole) break;  // uniform: every workgroup reaches this exit
        whole_tube<P, B, SUB>(a, item, F, G, C, s_bad);
    }
}

}  // namespace lbmx

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace {

lbm_status bfail(lbm_status s, const std::string &m) {
    lbmx::set_error(m.c_str());
    return s;
}

lbm_status bvalidate(const lbm_batch_desc *d) {
    if (!d) return bfail(LBM_EINVAL, "batch descriptor is NULL");
    if (d->abi_version != LBM_ABI_VERSION) return bfail(LBM_EINVAL, "abi_version mismatch");
    if (d->dtype != LBM_F32 && d->dtype != LBM_F64) return bfail(LBM_EINVAL, "dtype must be F32 or F64");
    if (d->num_instances < 1 || d->num_instances > (1 << 24))
        return bfail(LBM_EINVAL, "num_instances must be in [1, 2^24]");
    if (d->total_nodes < 4 * d->num_instances || d->total_nodes >= (1LL << 31))
        return bfail(LBM_EINVAL, "total_nodes must be >= 4 * num_instances and < 2^31");
    if (!d->offsets || !d->n_rot || !d->tau || !d->nsteps || !d->status || !d->workspace)
        return bfail(LBM_EINVAL, "device arrays must not be NULL");
    if (!d->f[0] || !d->f[1] || !d->g[0] || !d->g[1] || d->f[0] == d->f[1] || d->g[0] == d->g[1])
        return bfail(LBM_EINVAL, "population buffers must be non-NULL and distinct");
    if (d->block != 0 && d->block != 256 && d->block != 512 && d->block != 1024)
        return bfail(LBM_EINVAL, "block must be 0, 256, 512 or 1024");
    if (d->superstep < 0 || d->superstep > 128) return bfail(LBM_EINVAL, "superstep must be in [0, 128]");
    if (d->g_substeps < 0 || d->g_substeps > 64) return bfail(LBM_EINVAL, "g_substeps must be in [0, 64]");
    return LBM_OK;
}

struct Launch {
    int block, chunk, superstep, m, hw;
    size_t lds;
};

// Chunk-queue slots: twice the chunks of one pass over all long tubes, for
// any launch shape (a chunk covers >= 64 nodes, so a tube of L nodes has at
// most L / 64 + 1 chunks).
size_t queue_slots(const lbm_batch_desc *d) {
    return 2 * ((size_t)d->total_nodes / 64 + (size_t)d->num_instances);
}

// Chunk capacity: the largest multiple of 64 nodes whose two LDS buffers of
// 14 populations fit the LDS budget (at most `chunk` if given).
lbm_status plan(const lbm_batch_desc *d, Launch *L) {
    const int B = d->block ? d->block : (d->dtype == LBM_F32 ? 1024 : 512);
    const size_t sz = d->dtype == LBM_F32 ? 4 : 8;
    const size_t budget = 156 * 1024;
    int C = (int)(budget / (28 * sz)) / 64 * 64;
    if (d->chunk > 0) {
        if (d->chunk < 64) return bfail(LBM_EINVAL, "chunk must be >= 64");
        if (d->chunk / 64 * 64 < C) C = d->chunk / 64 * 64;
    }
    // A step reaches 3 nodes (streaming) and 2 m nodes (m rotational
    // advection sub-steps): chunk halos of hw nodes per step of a pass.
    const int m = d->g_substeps > 1 ? d->g_substeps : 1;
    const int hw = 2 * m > 3 ? 2 * m : 3;
    // Default passes of 128 / hw steps, at most 24: the halo recomputation
    // (2 hw S of C nodes) grows with m, the per-pass overhead with 1/S
    // (measured on the 4096-tube workload: m = 1: 24, m = 4: 16, m = 8: 8).
    int S = d->superstep ? d->superstep : std::max(4, std::min(24, 128 / hw));
    if (!d->superstep && C - 2 * hw * S < 64) S = (C - 64) / (2 * hw);
    if (S < 1 || C - 2 * hw * S < 64) return bfail(LBM_EINVAL, "superstep too large for the chunk");
    L->block = B;
    L->chunk = C;
    L->superstep = S;
    L->m = m;
    L->hw = hw;
    L->lds = 28 * sz * (size_t)C;
    return LBM_OK;
}

// prepare = true: raise the kernel's dynamic-LDS limit (outside capture);
// prepare = false: launch.
template <typename P, int B, bool SUB> hipError_t launch_batch_t(const lbmx::BatchArgs &a, size_t lds, int grid,
                                                                 hipStream_t s, bool prepare) {
    auto kern = lbmx::k_batch<P, B, SUB>;
    if (prepare)
        return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(B), lds, s, a);
    return hipGetLastError();
}

template <typename P, bool SUB> hipError_t launch_batch_ps(const Launch &L, const lbmx::BatchArgs &a, int grid,
                                                          hipStream_t s, bool prepare) {
    if (L.block == 256) return launch_batch_t<P, 256, SUB>(a, L.lds, grid, s, prepare);
    if (L.block == 512) return launch_batch_t<P, 512, SUB>(a, L.lds, grid, s, prepare);
    if (L.block == 1024) return launch_batch_t<P, 1024, SUB>(a, L.lds, grid, s, prepare);
    return hipErrorInvalidValue;
}
template <typename P> hipError_t launch_batch_p(const Launch &L, const lbmx::BatchArgs &a, int grid,
                                                hipStream_t s, bool prepare) {
    return L.m > 1 ? launch_batch_ps<P, true>(L, a, grid, s, prepare) : launch_batch_ps<P, false>(L, a, grid, s, prepare);
}

// Instantiated graphs of lbm_batch_step, keyed by the device and every
// descriptor field the recorded launches read; released by
// lbm_batch_release (or evicted oldest-first beyond kGraphCap entries).
struct GraphEntry {
    int dev;
    lbm_batch_desc d;
    hipGraphExec_t exec;
    hipEvent_t launched;  // recorded after every launch; waited for before the graph is destroyed
};

void destroy_entry(GraphEntry &en) {
    if (en.launched) {
        hipEventSynchronize(en.launched);
        hipEventDestroy(en.launched);
    }
    hipGraphExecDestroy(en.exec);
}
constexpr size_t kGraphCap = 16;
std::mutex g_mu;
std::vector<GraphEntry> g_cache;

bool same_desc(const lbm_batch_desc &x, const lbm_batch_desc &y) {
    return x.dtype == y.dtype && x.num_instances == y.num_instances &&
           x.total_nodes == y.total_nodes && x.offsets == y.offsets && x.n_rot == y.n_rot &&
           x.tau == y.tau && x.nsteps == y.nsteps && x.f[0] == y.f[0] && x.f[1] == y.f[1] &&
           x.g[0] == y.g[0] && x.g[1] == y.g[1] && x.status == y.status &&
           x.workspace == y.workspace && x.steps_done == y.steps_done && x.block == y.block && x.chunk == y.chunk &&
           x.superstep == y.superstep && x.g_substeps == y.g_substeps;
}

// Scratch of lbm_batch_step_noalloc: the workspace of the batched launch
// (schedule arrays, counters, chunk queue) in a fixed device array, for
// callers that cannot allocate.  Each device the library runs on holds its
// own copy until the process ends; its address on the current device comes
// from hipGetSymbolAddress (the array's name in host code is not a device
// address).
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scr_mu;
void *g_scr_ptr[kMaxDevices] = {};

lbm_status scratch_on_current_device(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return bfail(LBM_EDEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices) return bfail(LBM_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scr_mu);
    if (!g_scr_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return bfail(LBM_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
        g_scr_ptr[dev] = p;
    }
    *out = g_scr_ptr[dev];
    return LBM_OK;
}

hipError_t enqueue_batch(const lbm_batch_desc *d, const Launch &L, hipStream_t s, bool prepare) {
    lbmx::BatchArgs a;
    a.offsets = d->offsets;
    a.n_rot = d->n_rot;
    a.tau = d->tau;
    a.nsteps = d->nsteps;
    for (int k = 0; k < 2; ++k) {
        a.f[k] = d->f[k];
        a.g[k] = d->g[k];
    }
    a.status = d->status;
    a.steps_done = d->steps_done;
    const size_t n = (size_t)d->num_instances;
    a.counter = reinterpret_cast<int32_t *>(d->workspace);
    a.order = a.counter + lbmx::kCtrWords;
    a.ltube = a.order + n;
    a.lpas = a.ltube + n;
    a.lpfx = a.lpas + n;
    a.pdone = a.lpfx + n + 1;
    a.tpass = a.pdone + n;
    a.fail_at = reinterpret_cast<int64_t *>(a.counter + lbmx::kCtrWords + ((6 * n + 1 + 1) & ~(size_t)1));
    a.qcap = (int)queue_slots(d);
    a.qitem = a.fail_at + n;
    a.qseq = a.qitem + a.qcap;
    a.num = (int)d->num_instances;
    a.total = (uint32_t)d->total_nodes;
    a.chunk = L.chunk;
    a.superstep = L.superstep;
    a.m = L.m;
    a.hw = L.hw;
    int dev = 0, cus = 256;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // one workgroup per compute unit (the LDS chunk fills it): the long-tube
    // passes spread a tube's chunks over all of them
    const int grid = cus < lbmx::kMaxGrid ? cus : lbmx::kMaxGrid;
    if (!prepare) {
        hipLaunchKernelGGL(lbmx::k_batch_order, dim3(1), dim3(1024), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return d->dtype == LBM_F32 ? launch_batch_p<float>(L, a, grid, s, prepare)
                               : launch_batch_p<double>(L, a, grid, s, prepare);
}

}  // namespace

extern "C" {

size_t lbm_batch_workspace_bytes(const lbm_batch_desc *desc) {
    if (!desc || desc->num_instances < 1 || desc->total_nodes < 0) return 0;
    // counters [kCtrWords], order, ltube, lpas [n] each, lpfx [n+1], pdone,
    // tpass [n] each (int32, padded to 8 bytes); fail_at [n], chunk queue
    // items and sequences [queue_slots] each (int64)
    const size_t n = (size_t)desc->num_instances;
    const size_t i32 = lbmx::kCtrWords + ((6 * n + 1 + 1) & ~(size_t)1);
    return ((i32 * 4 + (n + 2 * queue_slots(desc)) * 8 + 255) / 256) * 256;
}

lbm_status lbm_batch_init(const lbm_batch_desc *desc, const double *rho, const double *u,
                          const double *T, void *hip_stream) {
    lbm_status st = bvalidate(desc);
    if (st) return st;
    if (!rho || !u || !T) return bfail(LBM_EINVAL, "rho, u, T must not be NULL");
    lbmx::InitArgs a{rho, u, T, desc->f[0], desc->g[0], (uint32_t)desc->total_nodes};
    hipError_t e = lbmx::launch_init(desc->dtype, 1, lbmx::kTensor, a, (hipStream_t)hip_stream);
    if (e != hipSuccess) return bfail(LBM_ELAUNCH, std::string("batch init: ") + hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_batch_step(const lbm_batch_desc *desc, void *hip_stream) {
    lbm_status st = bvalidate(desc);
    if (st) return st;
    Launch L;
    st = plan(desc, &L);
    if (st) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return bfail(LBM_EDEVICE, "hipGetDevice failed");
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &en : g_cache)
        if (en.dev == dev && same_desc(en.d, *desc)) {
            hipError_t e = hipGraphLaunch(en.exec, s);
            if (e != hipSuccess) return bfail(LBM_ELAUNCH, std::string("graph launch: ") + hipGetErrorString(e));
            if (en.launched) hipEventRecord(en.launched, s);
            return LBM_OK;
        }
    // record the order + persistent kernels once on a private stream
    hipError_t ep = enqueue_batch(desc, L, s, true);
    if (ep != hipSuccess) return bfail(LBM_ELAUNCH, std::string("batch LDS limit: ") + hipGetErrorString(ep));
    hipStream_t cap;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
        return bfail(LBM_EDEVICE, "stream create failed");
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = enqueue_batch(desc, L, cap, false);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cap, &graph);
    hipStreamDestroy(cap);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) hipGraphDestroy(graph);
        return bfail(LBM_ELAUNCH, std::string("batch capture: ") +
                                      hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) return bfail(LBM_ELAUNCH, std::string("graph instantiate: ") + hipGetErrorString(e));
    if (g_cache.size() >= kGraphCap) {
        destroy_entry(g_cache.front());
        g_cache.erase(g_cache.begin());
    }
    hipEvent_t launched = nullptr;
    if (hipEventCreateWithFlags(&launched, hipEventDisableTiming) != hipSuccess) launched = nullptr;
    g_cache.push_back({dev, *desc, exec, launched});
    e = hipGraphLaunch(exec, s);
    if (e != hipSuccess) return bfail(LBM_ELAUNCH, std::string("graph launch: ") + hipGetErrorString(e));
    if (launched) hipEventRecord(launched, s);
    return LBM_OK;
}

lbm_status lbm_batch_step_noalloc(const lbm_batch_desc *desc, void *hip_stream) {
    if (!desc) return bfail(LBM_EINVAL, "batch descriptor is NULL");
    lbm_batch_desc d = *desc;
    const size_t need = lbm_batch_workspace_bytes(&d);
    if (need > kNoAllocScratchBytes)
        return bfail(LBM_EINVAL, "batch needs " + std::to_string(need) + " bytes of scratch; the no-allocation "
                                 "entry point has " + std::to_string(kNoAllocScratchBytes));
    void *scr = nullptr;
    lbm_status st = scratch_on_current_device(&scr);
    if (st) return st;
    d.workspace = scr;
    st = bvalidate(&d);
    if (st) return st;
    Launch L;
    st = plan(&d, &L);
    if (st) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    // direct launches (no graph: instantiating one allocates); the schedule
    // kernel re-initialises every scratch word the persistent kernel reads
    hipError_t e = enqueue_batch(&d, L, s, true);
    if (e == hipSuccess) e = enqueue_batch(&d, L, s, false);
    if (e != hipSuccess) return bfail(LBM_ELAUNCH, std::string("batch launch: ") + hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_batch_release(const lbm_batch_desc *desc) {
    if (!desc) return bfail(LBM_EINVAL, "batch descriptor is NULL");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return bfail(LBM_EDEVICE, "hipGetDevice failed");
    std::lock_guard<std::mutex> lk(g_mu);
    for (size_t k = 0; k < g_cache.size();) {
        if (g_cache[k].dev == dev && same_desc(g_cache[k].d, *desc)) {
            destroy_entry(g_cache[k]);
            g_cache.erase(g_cache.begin() + (ptrdiff_t)k);
        } else {
            ++k;
        }
    }
    return LBM_OK;
}

lbm_status lbm_batch_moments(const lbm_batch_desc *desc, double *rho, double *u, double *T,
                             void *hip_stream) {
    lbm_status st = bvalidate(desc);
    if (st) return st;
    if (!rho && !u && !T) return LBM_OK;
    lbmx::FieldArgs a = {};
    a.f = desc->f[0];
    a.g = desc->g[0];
    a.n0 = (int)desc->total_nodes;
    a.n1 = 1;
    a.n2 = 1;
    a.N = (uint32_t)desc->total_nodes;
    a.layout = lbmx::kLayoutStreamed;  // the batch state is kept streamed
    a.n_rot = 0.0;
    a.rho = rho;
    a.u = u;
    a.T = T;
    a.offsets = desc->offsets;  // per-node n from the node's tube
    a.n_rot_inst = desc->n_rot;
    a.num_inst = (int)desc->num_instances;
    int nb = 0;
    hipError_t e = lbmx::launch_fields(desc->dtype, 1, lbmx::kTensor, a, &nb, (hipStream_t)hip_stream);
    if (e != hipSuccess) return bfail(LBM_ELAUNCH, std::string("batch moments: ") + hipGetErrorString(e));
    return LBM_OK;
}

}  // extern "C"
