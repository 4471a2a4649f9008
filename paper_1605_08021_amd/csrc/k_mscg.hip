// Multi-shift conjugate gradients for the compressed shifted equations of
// Eq. (3.6):  for one right-hand side b = -Q xi_mu and every Chebyshev shift,
//   (A + sigma_c I) z_c = b,   A = Q (H - s_base) Q,  sigma_c = s_base - s_c >= 0,
// where s_base is the shift closest to the LUMO (the slowest system).  The
// Krylov space of A + sigma I does not depend on sigma, so one CG sequence on A
// generates every shifted solution: the shifted residuals stay collinear,
// r_c = zeta_c r, and (Jegerlehner's recurrences)
//   zeta_{k+1} = zeta_k zeta_{k-1} a_{k-1} /
//                (a_k b_{k-1} (zeta_{k-1} - zeta_k) + zeta_{k-1} a_{k-1} (1 + sigma a_k))
//   a^c_k = a_k zeta_{k+1} / zeta_k,   b^c_k = b_k (zeta_{k+1} / zeta_k)^2
//   p_c <- zeta_k r_k + b^c_{k-1} p_c,   x_c += a^c_k p_c.
// Only the base sequence applies the stencil and the projector.  The vector
// updates of p_c and x_c (the base's x included) depend on the base residuals
// and on scalars only, so they are deferred: the residuals of a window of
// kMsWindow iterations stay in a ring, the step scalars in LDS, and once per
// window every p_c, x_c is read once, advanced through the window's steps in
// registers and written back.  That replaces 4 vector sweeps per shift and
// iteration by (4 per shift + the window's residuals) per window.
//
// Work decomposition (gfx950): a tile of 16 right-hand sides is shared by a
// group of K workgroups (8 waves each); workgroup k owns a contiguous range of
// 16-row blocks.  The base sequence runs CG in the Chronopoulos-Gear
// arrangement, so each iteration has a single reduction (Phi^T y, r.r, r.y):
// reduced inside each workgroup in LDS, then across the group through global
// memory behind a counter barrier; every workgroup sums the K partials in the
// same order, so all of them hold identical scalars.  The stencil's halo rows
// are exchanged through per-workgroup flags that only the neighbours wait for.
// The kernel is launched cooperatively, which guarantees that all workgroups
// of a group are resident; every wait is bounded and aborts the launch on
// expiry.
#include "krylov_common.h"

namespace acp {
namespace {

using namespace kry;

constexpr unsigned kSpinLimit = 1u << 22;   // ~seconds: a wait this long means a lost group
constexpr int MAXSH = 16;                   // shifts per right-hand side
constexpr int WS = kMsWindow;              // residual ring slots (longest window)
constexpr int WSLOTS = 8 * MAXSH;           // window step records per column: shifts x window
constexpr int KMAX = kMsMaxGroup;           // workgroups per tile

struct GroupSync {
    unsigned *cnt;      // barrier counter of this workgroup's (super-)group (monotonic)
    double *buf;        // per tile: [2 parities][K][slot]
    int slot;           // doubles per partial
    int K;
    int kg;
    unsigned members;   // workgroups that arrive at every barrier (K, or K SG in lockstep)
    unsigned phase;     // number of completed group barriers
    bool local;         // every workgroup of the group runs on this XCD (one L2)
};

// XCD (accelerator complex die) of the executing workgroup.
__device__ __forceinline__ unsigned xcd_id() {
    unsigned v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
    return v & 0xfu;
}

// This workgroup's partial buffer for the next group barrier.
__device__ __forceinline__ double *group_mine(const GroupSync &gs, int tile) {
    const size_t par = gs.phase & 1u;
    return gs.buf + (((size_t)tile * 2 + par) * gs.K + gs.kg) * (size_t)gs.slot;
}

// All threads, after writing this workgroup's partial to group_mine(): wait for
// the group and leave the ordered sum of the K partials (n doubles) in LDS dst.
// Returns false if the wait expired (the launch is then abandoned).
__device__ bool group_sum(GroupSync &gs, int tile, double *dst, int n, int *abort_flag) {
    const double *base = gs.buf + ((size_t)tile * 2 + (gs.phase & 1u)) * (size_t)gs.K * gs.slot;
    // every wave's stores complete before the barrier (the workgroup barrier
    // alone does not wait for global stores); thread 0's release then publishes
    // them
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    __shared__ int s_ok;
    if (threadIdx.x == 0) {
        // A group on one XCD shares one L2, through which every store of the
        // group passes (the vector L1 is write-through, and every wave waited
        // for its stores to complete before the barrier above): the counter
        // needs no L2 write-back on release, and acquiring needs only this
        // compute unit's L1 invalidated.  Otherwise the agent-scope
        // release/acquire pair.
        if (gs.local)
            __hip_atomic_fetch_add(gs.cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            __hip_atomic_fetch_add(gs.cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned target = (gs.phase + 1) * gs.members;
        unsigned spins = 0;
        int ok = 1;
        // spin on relaxed loads (an acquire per poll would invalidate caches every
        // time), then one acquire fence once the group has arrived
        while (__hip_atomic_load(gs.cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > kSpinLimit || __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                ok = 0;
                break;
            }
        }
        if (gs.local)
            asm volatile("buffer_inv sc0\n\ts_waitcnt vmcnt(0)" ::: "memory");   // L1 only
        else
            __atomic_thread_fence(__ATOMIC_ACQUIRE);   // agent scope (HIP's default for fences)
        if (!ok) __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_ok = ok;
    }
    // thread 0's acquire (same compute unit, so it also covers the other waves' reads)
    __syncthreads();
    gs.phase += 1;
    if (!s_ok) return false;
    // the K partials of two elements are loaded together (up to 2 KMAX loads in
    // flight per thread), then summed in group order
    const int K = gs.K;
    for (int i0 = threadIdx.x; i0 < n; i0 += 2 * NT) {
        const int i1 = i0 + NT < n ? i0 + NT : i0;
        double v0[KMAX], v1[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            if (k < K) {
                v0[k] = base[(size_t)k * gs.slot + i0];
                v1[k] = base[(size_t)k * gs.slot + i1];
            }
        }
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            if (k < K) {
                s0 += v0[k];
                s1 += v1[k];
            }
        }
        dst[i0] = s0;
        if (i0 + NT < n) dst[i1] = s1;
    }
    __syncthreads();
    return true;
}

// Column sums of a per-thread value (threads with equal t % 16), fixed order,
// written to out[0..15] (LDS or global).
__device__ __forceinline__ void column_partial(double v, double *red, double *out) {
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x < kTile) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NT / kTile; ++k) s += red[threadIdx.x + kTile * k];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// Halo exchange inside one tile's group: after writing its rows of a residual,
// a workgroup raises its flag to that residual's iteration number; before reading
// rows of the workgroups within D positions of it (cyclically) it waits until
// their flags reach that number.  Every wave first waits for its own stores, so
// the flag covers them; thread 0 then also refreshes this compute unit's L1,
// since the waves read each other's rows next.
__device__ __forceinline__ void halo_publish(const GroupSync &gs, int *flags, int k) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        if (gs.K > 1) {
            if (gs.local)
                __hip_atomic_store(flags + gs.kg, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else
                __hip_atomic_store(flags + gs.kg, k, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        asm volatile("buffer_inv sc0\n\ts_waitcnt vmcnt(0)" ::: "memory");
    }
    __syncthreads();
}

__device__ bool halo_wait(const GroupSync &gs, const int *flags, int D, int k, int *abort_flag) {
    __shared__ int s_hok;
    if (threadIdx.x == 0) {
        int ok = 1;
        for (int d = -D; d <= D && ok; ++d) {
            if (d == 0) continue;
            const int other = ((gs.kg + d) % gs.K + gs.K) % gs.K;
            unsigned spins = 0;
            while (__hip_atomic_load(flags + other, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < k) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > kSpinLimit ||
                    __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    break;
                }
            }
        }
        if (gs.local)
            asm volatile("buffer_inv sc0\n\ts_waitcnt vmcnt(0)" ::: "memory");
        else
            __atomic_thread_fence(__ATOMIC_ACQUIRE);
        if (!ok) __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_hok = ok;
    }
    __syncthreads();
    return s_hok != 0;
}

// Column sums of two per-thread values (fixed order), to out[0..15] and out[16..31].
__device__ __forceinline__ void column_partial2(double v0, double v1, double *red, double *out) {
    red[threadIdx.x] = v0;
    red[NT + threadIdx.x] = v1;
    __syncthreads();
    if (threadIdx.x < 2 * kTile) {
        const int h = threadIdx.x / kTile, c = threadIdx.x % kTile;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NT / kTile; ++k) s += red[h * NT + c + kTile * k];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

#ifdef ACP_PHASE_CLOCKS
// Per-phase timers of workgroup 0, thread 0 (tuning builds only).
#define PHASE_MARK(i)                                                          \
    do {                                                                       \
        if (prof) {                                                            \
            const unsigned long long now_ = wall_clock64();                    \
            prof_acc[i] += now_ - prof_last;                                   \
            prof_last = now_;                                                  \
        }                                                                      \
    } while (0)
#else
#define PHASE_MARK(i) do {} while (0)
#endif

// The whole solve of one right-hand-side tile (all shifts) by workgroup kg of
// its group.  The base sequence is CG in the Chronopoulos-Gear arrangement,
//   r_{k+1} = r_k - a_k s_k,   w = A r_{k+1},
//   g_{k+1} = r.r,  d_{k+1} = r.w,  b_k = g_{k+1} / g_k,
//   a_{k+1} = g_{k+1} / (d_{k+1} - b_k g_{k+1} / a_k),   s_{k+1} = w + b_k s_k,
// which yields the scalars of textbook CG (a_k, b_k, with p_k^T A p_k =
// d_k - b_{k-1} g_k / a_{k-1}) from one reduction per iteration: C = Phi^T y,
// r.r and r.y (= r.w, as r lies in range(Q)) travel together.  Workgroup kg owns
// a contiguous range of 16-row blocks; between the sweep that writes r_{k+1} and
// the sweep that applies the stencil to it, only the stencil neighbours' rows
// are awaited (per-workgroup flags), and the blocks away from the range ends
// are processed first.
template <int DIM, int NB, typename T>
__device__ void mscg_tile(const MsArgsT<T> &a, const int tile, const int kg) {
    using S = Slots<NB>;
    static_assert(S::N * S::ELEMS >= S::ELEMS + 2 * kTile, "slots hold C, r.r and r.y");
    __shared__ double slots[S::N * S::ELEMS];
    __shared__ double red[2 * NT];
    __shared__ double s_rr[kTile], s_bn[kTile], s_al[kTile], s_btp[kTile], s_alp[kTile],
        s_tmp[kTile];
    __shared__ double s_z[MAXSH][kTile], s_zp[MAXSH][kTile], s_bs[MAXSH][kTile],
        s_res[MAXSH][kTile];
    // step scalars of the current window: p = wz r + wb p, x += wa p
    // (record of shift c, step w at c * wl + w; windows of wl = 16 steps when
    // there are at most 8 shifts, else 8)
    __shared__ double s_wz[WSLOTS][kTile], s_wb[WSLOTS][kTile], s_wa[WSLOTS][kTile];
    __shared__ int s_act[MAXSH][kTile], s_it[MAXSH][kTile], s_wn[MAXSH][kTile], s_flag[kTile],
        s_colact[kTile], s_any, s_abort;

    const int K = a.K;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int col = lane & 15;
    const int q = lane >> 4;
    const int ns = a.nshift;
    const int bs = a.base;
    const int wl = ns <= 8 ? 16 : 8;   // window length (wl * ns <= WSLOTS)
    const int ng = a.g.ng;
    const long long tstride = (long long)ng * kTile;
    const T *__restrict__ b = a.rhs + (long long)tile * tstride;
    T *sv = a.pa + (long long)tile * tstride;   // s = A p of the base sequence (own rows)
    int *hflags = a.hflag ? a.hflag + (size_t)tile * K : nullptr;
    // shift c of this tile: X[c] at a.x + (c * ntiles + tile) * tstride, same for P;
    // residual of iteration k at ring slot k % WS
    auto Xs = [&](int c) { return a.x + ((long long)c * a.ntiles + tile) * tstride; };
    auto Ps = [&](int c) { return a.p + ((long long)c * a.ntiles + tile) * tstride; };
    auto Rs = [&](int k) { return a.r + ((long long)(k % WS) * a.ntiles + tile) * tstride; };
    const double sbase = a.shift[bs];
    // lockstep: the SG tiles tile mod (ntiles / SG) share one barrier counter
    // (and then one XCD, which makes them read the same rows of Phi at about
    // the same time); every other use of the group stays per tile
    const int SG = a.sg > 1 ? a.sg : 1;
    const int nsg = a.ntiles / SG;
    const int sgid = tile % nsg;
    GroupSync gs{a.cnt + (SG > 1 ? sgid : tile), a.gbuf, S::ELEMS + 2 * kTile, K, kg,
                 (unsigned)(K * SG), 0u, false};
    const int nblk = (ng + 15) / 16;
    // this workgroup's blocks [kb0, kb1) and rows [r0, r1)
    const int kb0 = (int)((long long)kg * nblk / K), kb1 = (int)((long long)(kg + 1) * nblk / K);
    const int r0 = kb0 * 16, r1 = kb1 * 16 < ng ? kb1 * 16 : ng;
    const int own_rows = (kb1 - kb0) * 16;
    // stencil reach in grid rows, the neighbours within it, and the blocks whose
    // stencil leaves the range
    const int reach = DIM == 1 ? 4 : 4 * a.g.nx;
    const int min_chunk = (nblk / K) * 16;
    const int D = K == 1 ? 0 : (min_chunk > 0 ? min((reach + min_chunk - 1) / min_chunk, K - 1) : K - 1);
    auto boundary = [&](int blk) {
        return K > 1 && (blk * 16 - reach < r0 || blk * 16 + 16 + reach > r1);
    };

#ifdef ACP_PHASE_CLOCKS
    const bool prof = a.phase_clock && blockIdx.x == 0 && t == 0;
    unsigned long long prof_acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    unsigned long long prof_last = prof ? wall_clock64() : 0ull;
#endif

    // Deferred updates of the window that started at iteration k0 (n_steps
    // steps, uniform over the group): every thread walks this workgroup's rows
    // for system j = t % 16, four rows at a time, and for every shift with
    // recorded steps reads p_c, x_c once, applies the steps and writes them back.
    // The next shift's loads are issued before the current shift's arithmetic.
    auto flush = [&](int k0, int n_steps) {
        const int j = t & 15;
        constexpr int RR = 2;
        constexpr int RSTEP = NT / kTile;
        for (int rl0 = t >> 4; rl0 < own_rows; rl0 += RR * RSTEP) {
            long long id[RR];
            bool ok[RR];
#pragma unroll
            for (int i = 0; i < RR; ++i) {
                const int rl = rl0 + i * RSTEP;
                const int row = r0 + rl;
                ok[i] = rl < own_rows && row < ng;
                id[i] = (long long)(ok[i] ? row : 0) * kTile + j;   // row 0 always exists
            }
            double rw[WS][RR];
#pragma unroll
            for (int w = 0; w < WS; ++w) {
                if (w < n_steps) {
                    const T *rk = Rs(k0 + w);
#pragma unroll
                    for (int i = 0; i < RR; ++i) rw[w][i] = (double)rk[id[i]];
                }
            }
            double pn[RR] = {}, xn[RR] = {};
            int nn = s_wn[0][j];
            if (nn > 0) {
#pragma unroll
                for (int i = 0; i < RR; ++i) {
                    pn[i] = (double)Ps(0)[id[i]];
                    xn[i] = Xs(0)[id[i]];
                }
            }
            for (int c = 0; c < ns; ++c) {
                const int n = nn;
                double pv[RR], xv[RR];
#pragma unroll
                for (int i = 0; i < RR; ++i) {
                    pv[i] = pn[i];
                    xv[i] = xn[i];
                }
                if (c + 1 < ns) {
                    nn = s_wn[c + 1][j];
                    if (nn > 0) {
#pragma unroll
                        for (int i = 0; i < RR; ++i) {
                            pn[i] = (double)Ps(c + 1)[id[i]];
                            xn[i] = Xs(c + 1)[id[i]];
                        }
                    }
                }
                if (n > 0) {
#pragma unroll
                    for (int w = 0; w < WS; ++w) {
                        if (w < n) {
                            const int wi = c * wl + w;
                            const double wz = s_wz[wi][j], wb = s_wb[wi][j], wa = s_wa[wi][j];
#pragma unroll
                            for (int i = 0; i < RR; ++i) {
                                pv[i] = wb * pv[i] + wz * rw[w][i];
                                xv[i] += wa * pv[i];
                            }
                        }
                    }
                    T *pc = Ps(c);
                    double *xc = Xs(c);
#pragma unroll
                    for (int i = 0; i < RR; ++i)
                        if (ok[i]) {
                            pc[id[i]] = (T)pv[i];
                            xc[id[i]] = xv[i];
                        }
                }
            }
        }
        __syncthreads();
        if (t < kTile * MAXSH) s_wn[t / kTile][t % kTile] = 0;
        __syncthreads();
    };

    if (t == 0) s_abort = 0;
    // ---- init (own rows): r_0 = b, s = 0, x_c = 0, p_c = 0; |b|^2 (a resumed
    // tile finds its vectors in place)
    const bool resume = a.it0 > 0;
    double bb = 0.0;
    if (!resume) {
        T *rz = Rs(0);
        for (int blk = kb0 + wave; blk < kb1; blk += NW) {
            const int R = blk * 16 + 4 * q;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = R + j;
                if (row < ng) {
                    const int id = row * kTile + col;
                    const double bv = (double)b[id];
                    rz[id] = (T)bv;
                    sv[id] = (T)0.0;
                    for (int c = 0; c < ns; ++c) {
                        Xs(c)[id] = 0.0;
                        Ps(c)[id] = (T)0.0;
                    }
                    bb += bv * bv;
                }
            }
        }
    }
    // the first barrier (agent scope) also publishes each workgroup's XCD and
    // makes r_0 visible to the whole group
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __shared__ int s_local;
    {
        double *mine = group_mine(gs, tile);
        if (t == 0) mine[kTile] = (double)xcd_id();
        column_partial(bb, red, mine);
    }
    if (!group_sum(gs, tile, s_tmp, kTile, a.abort_flag)) return;
    if (t == 0) {
        // every workgroup that shares the barrier counter on this XCD?
        const double me = (double)xcd_id();
        int same = 1;
        for (int j = 0; j < SG; ++j) {
            const double *first = a.gbuf + (size_t)(sgid + j * nsg) * 2 * K * gs.slot;   // parity 0
            for (int k = 0; k < K; ++k) same &= first[(size_t)k * gs.slot + kTile] == me;
        }
        s_local = same;
        asm volatile("buffer_inv sc0\n\ts_waitcnt vmcnt(0)" ::: "memory");
    }
    __syncthreads();
    gs.local = s_local != 0;
    // scalar state of a resumed tile, as the suspending launch left it
    auto st_at = [&](int f) -> double & {
        return a.state[((size_t)tile * kMsStateFields + f) * kTile + t];
    };
    if (resume && t < kTile) {
        s_rr[t] = st_at(0);
        s_bn[t] = st_at(1);
        s_btp[t] = st_at(2);
        s_alp[t] = st_at(3);
        s_flag[t] = (int)st_at(4);
        s_colact[t] = (int)st_at(5);
        for (int c = 0; c < ns; ++c) {
            s_z[c][t] = st_at(8 + 6 * c);
            s_zp[c][t] = st_at(9 + 6 * c);
            s_bs[c][t] = st_at(10 + 6 * c);
            s_res[c][t] = st_at(11 + 6 * c);
            s_act[c][t] = (int)st_at(12 + 6 * c);
            s_it[c][t] = (int)st_at(13 + 6 * c);
        }
    } else if (t < kTile) {
        const double bn = sqrt(s_tmp[t]);
        s_bn[t] = bn;
        s_rr[t] = s_tmp[t];
        s_alp[t] = 1.0;
        s_btp[t] = 0.0;
        s_flag[t] = 0;
        for (int c = 0; c < ns; ++c) {
            s_z[c][t] = 1.0;
            s_zp[c][t] = 1.0;
            s_bs[c][t] = 0.0;
            s_res[c][t] = -1.0;
            s_act[c][t] = bn > 0.0 ? 1 : 0;
            s_it[c][t] = 0;
        }
    }
    if (t < kTile * MAXSH) s_wn[t / kTile][t % kTile] = 0;
    __syncthreads();

    constexpr int nep = NB * 16;
    constexpr int NN = Nbr<DIM>::N;
    int it = a.it0, k0 = a.it0;
    bool suspended = false;
    for (;;) {
        // suspension at a window boundary (k0 == it: no deferred steps pending)
        if (it == a.stop_at && it > a.it0) {
            suspended = true;
            break;
        }
        const T *rcur = Rs(it);
        // ---- sweep B: y = (H - s_base) r_it, C = Phi^T y, r.r, r.y; blocks away
        // from the range ends first, then (neighbours' rows of r_it awaited) the rest
        d4 acc[NB];
#pragma unroll
        for (int mb = 0; mb < NB; ++mb) acc[mb] = d4{0.0, 0.0, 0.0, 0.0};
        double gam = 0.0, del = 0.0;
        auto sweep_b = [&](bool ends) {
            for (int blk = kb0 + wave; blk < kb1; blk += NW) {
                if (boundary(blk) != ends) continue;
                const int R = blk * 16 + 4 * q;
                const Nbr<DIM> nb(R, a.g);
                double w[NN];
#pragma unroll
                for (int k = 0; k < NN; ++k) w[k] = (double)rcur[nb.idx[k] * kTile + col];
                double av[4][NB];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = R + j < ng ? R + j : ng - 1;
                    const T *ph = a.phi_rm + (long long)row * nep + col;
#pragma unroll
                    for (int mb = 0; mb < NB; ++mb) av[j][mb] = (double)ph[mb * 16];
                }
                double y[4], rc[4];
                stencil_from<DIM>(w, R, a.g, a.veff, sbase, y, rc);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    gam += rc[j] * rc[j];
                    del += rc[j] * y[j];
                }
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int mb = 0; mb < NB; ++mb)
                        acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j][mb], y[j], acc[mb], 0, 0, 0);
            }
        };
        sweep_b(false);
        if (K > 1 && it > 0 && !halo_wait(gs, hflags, D, it, a.abort_flag)) {
            if (t == 0) s_abort = 1;
            break;
        }
        sweep_b(true);
        PHASE_MARK(0);
        // workgroup reduction of C through the LDS slots (fixed order), published
        // with r.r and r.y as this workgroup's partial
#pragma unroll 1
        for (int ph = 0; ph < NW / S::N; ++ph) {
            if (wave / S::N == ph) {
                double *dst = slots + (wave % S::N) * S::ELEMS;
#pragma unroll
                for (int mb = 0; mb < NB; ++mb)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int idx = (mb * 16 + q + 4 * e) * kTile + col;
                        if (ph == 0) dst[idx] = acc[mb][e];
                        else dst[idx] += acc[mb][e];
                    }
            }
            __syncthreads();
        }
        {
            double *mine = group_mine(gs, tile);
            for (int idx = t; idx < S::ELEMS; idx += NT) {
                double v = slots[idx];
#pragma unroll
                for (int k = 1; k < S::N; ++k) v += slots[k * S::ELEMS + idx];
                mine[idx] = v;
            }
            column_partial2(gam, del, red, mine + S::ELEMS);
        }
        PHASE_MARK(1);
        // group reduction: slots[0..ELEMS) = C, then r.r, then r.y
        if (!group_sum(gs, tile, slots, S::ELEMS + 2 * kTile, a.abort_flag)) {
            if (t == 0) s_abort = 1;
            break;
        }
        PHASE_MARK(2);
        const double *g_rr = slots + S::ELEMS, *g_ry = slots + S::ELEMS + kTile;
        if (it > 0) {
            // convergence of r_it and the shifted b^c_{it-1}
            if (t < kTile * ns) {
                const int c = t / kTile, j = t % kTile;
                const double rrn = g_rr[j];
                const double bt = (s_rr[j] > 0.0) ? rrn / s_rr[j] : 0.0;
                const double thr = a.tol * s_bn[j];
                if (c == bs) {
                    if (s_act[c][j]) {
                        s_it[c][j] = it;
                        if (sqrt(rrn) <= thr) s_act[c][j] = 0;
                    }
                } else if (s_act[c][j]) {
                    const double zr = s_z[c][j] / s_zp[c][j];
                    const double res = fabs(s_z[c][j]) * sqrt(rrn);
                    s_bs[c][j] = bt * zr * zr;
                    s_it[c][j] = it;
                    if (res <= thr) {
                        s_act[c][j] = 0;
                        s_res[c][j] = res / s_bn[j];
                    }
                }
            }
            __syncthreads();
            if (t < kTile && s_colact[t]) {
                s_btp[t] = (s_rr[t] > 0.0) ? g_rr[t] / s_rr[t] : 0.0;
                s_rr[t] = g_rr[t];
            }
        }
        // a right-hand side whose shifts have all converged stops its base sequence too
        if (t < kTile) {
            int ca = 0;
            for (int c = 0; c < ns; ++c) ca |= s_act[c][t];
            s_colact[t] = ca;
            if (!ca) s_btp[t] = 0.0;
        }
        __syncthreads();
        if (t == 0) {
            int any = 0;
            for (int j = 0; j < kTile; ++j) any |= s_colact[j];
            s_any = any;
        }
        __syncthreads();
        if (!s_any || it >= a.max_iter) break;
        // base step a_it = g / (p^T A p), p^T A p = d - b_{it-1} g / a_{it-1}; a
        // non-positive curvature stops that right-hand side and is reported
        if (t < kTile) {
            double al = 0.0;
            if (s_colact[t]) {
                const double gg = s_rr[t];
                const double pap = it == 0 ? g_ry[t] : g_ry[t] - s_btp[t] * gg / s_alp[t];
                if (pap > 0.0) {
                    al = gg / pap;
                } else {
                    // with FP32 storage the rearranged curvature can lose its sign
                    // to storage rounding late in the solve: the column stops
                    // unconverged and the FP64 refinement finishes it
                    s_flag[t] |= sizeof(T) == 4 ? 1 : 2;
                    s_colact[t] = 0;
                }
            }
            s_al[t] = al;
        }
        __syncthreads();
        // the step of this iteration for every live sequence: zeta_{k+1} and a^c_k
        // of each active shift; the base (zeta = 1) keeps stepping while any shift
        // of its right-hand side is active
        {
            const int wpos = it - k0;
            if (t < kTile * ns) {
                const int c = t / kTile, j = t % kTile;
                const double al = s_al[j];
                if (!s_colact[j]) {
                    s_act[c][j] = 0;
                } else if (c == bs) {
                    s_wz[c * wl + wpos][j] = 1.0;
                    s_wb[c * wl + wpos][j] = s_btp[j];
                    s_wa[c * wl + wpos][j] = al;
                    s_wn[c][j] = wpos + 1;
                } else if (s_act[c][j]) {
                    const double sig = sbase - a.shift[c];
                    const double zk = s_z[c][j], zkm = s_zp[c][j];
                    const double alp = s_alp[j], btp = s_btp[j];
                    const double den = al * btp * (zkm - zk) + zkm * alp * (1.0 + sig * al);
                    const double zn = (den != 0.0) ? zk * zkm * alp / den : 0.0;
                    s_wz[c * wl + wpos][j] = zk;
                    s_wb[c * wl + wpos][j] = s_bs[c][j];
                    s_wa[c * wl + wpos][j] = (zk != 0.0) ? al * zn / zk : 0.0;
                    s_wn[c][j] = wpos + 1;
                    s_zp[c][j] = zk;
                    s_z[c][j] = zn;
                }
            }
            __syncthreads();
            // window full: apply it before the sweep below overwrites its oldest residual
            if (wpos == wl - 1) {
                flush(k0, wl);
                k0 = it + 1;
            }
        }
        PHASE_MARK(3);
        // ---- sweep CA: w = y - Phi C (= A r_it), s = w + b_{it-1} s,
        // r_{it+1} = r_it - a_it s (next ring slot)
        {
            const double al = s_al[col], beta = s_btp[col];
            T *rnext = Rs(it + 1);
            for (int blk = kb0 + wave; blk < kb1; blk += NW) {
                const int row0 = blk * 16;
                const int R = row0 + 4 * q;
                double w[NN];
                gather<DIM>(rcur, R, a.g, col, w);
                double so[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = R + e < ng ? R + e : ng - 1;
                    so[e] = (double)sv[row * kTile + col];
                }
                const d4 d = project_block<NB, T>(a.phi_cm, ng, slots, row0);
                double y[4], rc[4];
                stencil_from<DIM>(w, R, a.g, a.veff, sbase, y, rc);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double sn = (y[e] - d[e]) + beta * so[e];
                    const double rn = rc[e] - al * sn;
                    if (R + e < ng) {
                        sv[(R + e) * kTile + col] = (T)sn;
                        rnext[(R + e) * kTile + col] = (T)rn;
                    }
                }
            }
        }
        PHASE_MARK(4);
        halo_publish(gs, hflags, it + 1);
        if (t < kTile && s_colact[t]) s_alp[t] = s_al[t];
        __syncthreads();
        PHASE_MARK(5);
        ++it;
    }
#ifdef ACP_PHASE_CLOCKS
    if (prof)
        for (int i = 0; i < 8; ++i) a.phase_clock[i] = prof_acc[i];
#endif
    if (s_abort) return;
    // the partial last window
    if (it > k0) flush(k0, it - k0);
    if (kg == 0 && t < kTile * ns) {
        const int c = t / kTile, j = t % kTile;
        const long long gcol = ((long long)c * a.ntiles + tile) * kTile + j;
        a.iters[gcol] = s_it[c][j];
        double res;
        if (c != bs && s_res[c][j] >= 0.0) res = s_res[c][j];   // converged shift
        else {
            const double zc = (c == bs) ? 1.0 : fabs(s_z[c][j]);
            res = (s_bn[j] > 0.0) ? zc * sqrt(s_rr[j]) / s_bn[j] : 0.0;
        }
        a.resid[gcol] = res;
        a.flags[gcol] = s_flag[j] | (s_act[c][j] ? 1 : 0);
    }
    if (kg == 0 && t == 0) a.tile_iters[tile] = it;
    if (a.state && kg == 0 && t < kTile) {
        st_at(6) = suspended ? 1.0 : 0.0;
        // right-hand sides to carry into the next launch, after every tile's state
        a.state[((size_t)a.ntiles * kMsStateFields + tile) * kTile + t] =
            suspended && s_colact[t] ? 1.0 : 0.0;
        if (suspended) {
            st_at(0) = s_rr[t];
            st_at(1) = s_bn[t];
            st_at(2) = s_btp[t];
            st_at(3) = s_alp[t];
            st_at(4) = (double)s_flag[t];
            st_at(5) = (double)s_colact[t];
            for (int c = 0; c < ns; ++c) {
                st_at(8 + 6 * c) = s_z[c][t];
                st_at(9 + 6 * c) = s_zp[c][t];
                st_at(10 + 6 * c) = s_bs[c][t];
                st_at(11 + 6 * c) = s_res[c][t];
                st_at(12 + 6 * c) = (double)s_act[c][t];
                st_at(13 + 6 * c) = (double)s_it[c][t];
            }
        }
    }
    if (SG > 1) {
        // lockstep: keep arriving at the shared barrier until every tile of the
        // super-group is done (the last one to finish brings the count to zero
        // before its next arrival, so all leave after the same barrier)
        if (t == 0 && kg == 0) {
            __hip_atomic_fetch_add(a.active + sgid, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        }
        for (;;) {
            if (!group_sum(gs, tile, s_tmp, 0, a.abort_flag)) return;
            if (t == 0) s_any = __hip_atomic_load(a.active + sgid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            const int left = s_any;
            __syncthreads();
            if (left == 0) break;
        }
    }
}

// Group members blockIdx = tile + ntiles * k: with workgroups dealt round-robin
// to the XCDs, a group whose ntiles is a multiple of the XCD count stays on one
// XCD (one L2) for its barriers and halo exchange.
template <int DIM, int NB, typename T>
__global__ __launch_bounds__(NT) void mscg_kernel(MsArgsT<T> a) {
    mscg_tile<DIM, NB, T>(a, blockIdx.x % a.ntiles, blockIdx.x / a.ntiles);
}

// Persistent batch: every workgroup takes the next entry of a work list (one
// member kg of the group of one right-hand-side tile of one system, coded as
// tile * KMAX + kg) from a global counter until the list is exhausted; systems
// of different sizes (and group sizes, systems[s].K) share the launch.  The K
// members of a group are consecutive entries and the counter hands entries out
// in order, so at most one group is ever incomplete, and its missing members
// are the next entries taken by workgroups that finish complete groups: with a
// grid of at least K resident workgroups every group barrier is reached.
template <int DIM, int NB, typename T>
__global__ __launch_bounds__(NT) void mscg_batch_kernel(const MsArgsT<T> *__restrict__ systems,
                                                        const int *__restrict__ work_sys,
                                                        const int *__restrict__ work_tile, int n_work,
                                                        unsigned *queue) {
    __shared__ int s_w;
    for (;;) {
        __syncthreads();   // the previous entry is finished with s_w and the LDS state
        if (threadIdx.x == 0)
            s_w = (int)__hip_atomic_fetch_add(queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int w = s_w;
        if (w >= n_work) break;
        const MsArgsT<T> a = systems[work_sys[w]];
        mscg_tile<DIM, NB, T>(a, work_tile[w] / KMAX, work_tile[w] % KMAX);
    }
}

template <int DIM, int NB, typename T>
hipError_t launch_ms(const MsArgsT<T> &a, hipStream_t s) {
    MsArgsT<T> args = a;
    void *kargs[] = {&args};
    return hipLaunchCooperativeKernel((const void *)mscg_kernel<DIM, NB, T>,
                                      dim3(a.ntiles * a.K), dim3(NT), kargs, 0, s);
}

template <int DIM, int NB, typename T>
int max_groups_resident() {
    int nb = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)mscg_kernel<DIM, NB, T>, NT, 0) !=
        hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return nb * cus;
}

}  // namespace

#define ACP_NB_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

int mscg_resident_capacity(int dim, int ne, bool fp32) {
    const int nb = (ne + 15) / 16;
#define CASE(N)                                                                            \
    if (nb == N) {                                                                         \
        if (fp32) return dim == 1 ? max_groups_resident<1, N, float>() : max_groups_resident<2, N, float>(); \
        return dim == 1 ? max_groups_resident<1, N, double>() : max_groups_resident<2, N, double>(); \
    }
    ACP_NB_CASES(CASE)
#undef CASE
    return 0;
}

size_t mscg_group_slot(int ne) {
    const int nb = (ne + 15) / 16;
    return (size_t)nb * 16 * kTile + 2 * kTile;
}

template <typename T>
hipError_t launch_mscg(const MsArgsT<T> &a, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    if (a.nshift > MAXSH || a.ne > 256 || a.K < 1 || a.K > KMAX) return hipErrorInvalidValue;
    const int nb = (a.ne + 15) / 16;
    // 2D grids whose lines hold a multiple of 4 points take the compact stencil
    // gather (the 4 rows of a group share one line)
    const bool compact2d = a.g.dim == 2 && a.g.nx % 4 == 0;
#define CASE(N)                                                                    \
    if (nb == N)                                                                   \
        return a.g.dim == 1 ? launch_ms<1, N, T>(a, s)                             \
                            : compact2d ? launch_ms<3, N, T>(a, s) : launch_ms<2, N, T>(a, s);
    ACP_NB_CASES(CASE)
#undef CASE
    return hipErrorInvalidValue;
}

hipError_t launch_mscg_fp64(const MsArgs &a, hipStream_t s) { return launch_mscg(a, s); }

hipError_t launch_mscg_batch_fp64(int dim, int ne_pad, const MsArgs *systems, const int *work_sys,
                                  const int *work_tile, int n_work, unsigned *queue, int grid,
                                  hipStream_t s) {
    if (n_work <= 0) return hipSuccess;
    if (grid < 1 || ne_pad > 256) return hipErrorInvalidValue;
    const int nb = (ne_pad + 15) / 16;
#define CASE(N)                                                                                      \
    if (nb == N) {                                                                                   \
        if (dim == 1)                                                                                \
            hipLaunchKernelGGL((mscg_batch_kernel<1, N, double>), dim3(grid), dim3(NT), 0, s, systems, \
                               work_sys, work_tile, n_work, queue);                                  \
        else if (dim == 3)                                                                           \
            hipLaunchKernelGGL((mscg_batch_kernel<3, N, double>), dim3(grid), dim3(NT), 0, s, systems, \
                               work_sys, work_tile, n_work, queue);                                  \
        else                                                                                         \
            hipLaunchKernelGGL((mscg_batch_kernel<2, N, double>), dim3(grid), dim3(NT), 0, s, systems, \
                               work_sys, work_tile, n_work, queue);                                  \
        return hipGetLastError();                                                                    \
    }
    ACP_NB_CASES(CASE)
#undef CASE
    return hipErrorInvalidValue;
}
hipError_t launch_mscg_fp32(const MsArgsT<float> &a, hipStream_t s) { return launch_mscg(a, s); }

}  // namespace acp
