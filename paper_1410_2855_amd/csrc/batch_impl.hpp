// batch_impl.hpp -- kernels that advance many cavities together: the grouped
// passes (one launch per pass: k_pass, and its software-pipelined form
// k_pass_pipe) and the persistent round-trip kernel k_trip described here.
//
// k_trip: all cavities of a group advance one round trip per launch.  The work of a
// trip is a list of tasks (row blocks and column blocks of every cavity),
// ordered by the host packer so that a cavity's column tasks come after all
// of its row tasks.  Workgroups take tickets from an atomic queue in chunks
// and run the tasks in ticket order; a column task first waits until its
// cavity's row-done counter reaches the number of row blocks (release on the
// producer side, acquire on the consumer side, both at device scope since
// the eight XCDs have separate L2 caches).  Because a column task only ever
// waits on tickets smaller than its own, which running workgroups hold and
// finish without waiting, the queue cannot deadlock for any grid size.  The
// wait is still bounded: after ~2 s it raises an abort flag that releases
// every waiter, and the cavity's counters report the failure to the host.  The
// last workgroup to leave resets the queue head and the counters, so the same
// launch can be replayed from a HIP graph.
#pragma once

#include <hip/hip_ext.h>

#include <initializer_list>

#include "batch.hpp"
#include "map.hpp"

namespace lsr {

// Reset a queue counter with an atomic read-modify-write (returns the old value).
__device__ __forceinline__ unsigned atomic_zero(unsigned* p) {
    return __hip_atomic_exchange(p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sizes sharing one persistent kernel: same workgroup size; the LDS buffer
// is the largest of their line buffers.
template <class S0, class... Ss>
struct Group {
    static constexpr int THREADS = S0::THREADS;
    static_assert(((Ss::THREADS == THREADS) && ...), "one group, one workgroup size");
    static constexpr int maxl() {
        int m = S0::LDS_ELEMS * 8;
        ((m = m > Ss::LDS_ELEMS * 8 ? m : Ss::LDS_ELEMS * 8), ...);
        return m;
    }
};

// ANY = 0: the default local step, compiled in; ANY = 1: the cavity's own
// local-step model (d.model, uniform in a workgroup), one compiled body each;
// ANY = 2: also the roughness bodies (groups holding a rough cavity; the
// batch puts no rough cavity in the others).  ANY = ANY_FIXED + m: model m
// alone, compiled in (groups whose cavities all have model m and a smooth
// mirror; no switch, so no registers of the other bodies).
// Kernels that read each cavity's code (ANY = 1, 2) also take a cavity's
// general transfer function (prop_kind 2, the map with kernel K of Eq. (10))
// in their column tasks: a uniform branch per task.
template <int ANY>
constexpr bool takes_trans() { return ANY == 1 || ANY == 2; }

template <int MODE, int ANY, class S>
__device__ __forceinline__ bool run_if(const CavDesc& d, int kind, int blk, unsigned char* smem, double* red) {
    if (d.N != S::N) return false;
    cx<float>* lds = reinterpret_cast<cx<float>*>(smem);
    if (kind == TASK_ROW) {
        if constexpr (ANY >= ANY_FIXED && MODE != ROW_LAST) {
            row_task<S, float, MODE, ANY - ANY_FIXED>(d, blk, lds, red);
        } else if constexpr (ANY && MODE != ROW_LAST) {
            switch (d.model) {
            case 1: row_task<S, float, MODE, 1>(d, blk, lds, red); break;
            case 2: row_task<S, float, MODE, 2>(d, blk, lds, red); break;
            case MODEL_ROUGH + 0:
                if constexpr (ANY == 2) row_task<S, float, MODE, MODEL_ROUGH + 0>(d, blk, lds, red);
                break;
            case MODEL_ROUGH + 1:
                if constexpr (ANY == 2) row_task<S, float, MODE, MODEL_ROUGH + 1>(d, blk, lds, red);
                break;
            case MODEL_ROUGH + 2:
                if constexpr (ANY == 2) row_task<S, float, MODE, MODEL_ROUGH + 2>(d, blk, lds, red);
                break;
            default: row_task<S, float, MODE, 0>(d, blk, lds, red); break;
            }
        } else {
            row_task<S, float, MODE>(d, blk, lds, red);
        }
    } else if (takes_trans<ANY>() && d.prop_kind == 2) {
        col_task<S, float, COL_PROP, PROP_TRANS>(d, blk, lds);
    } else {
        col_task<S, float, COL_PROP>(d, blk, lds);
    }
    return true;
}

// WPE: waves per SIMD the register allocation must allow (4 leaves 128
// VGPRs, 2 leaves 256); the autotuner picks the faster variant.  The row
// kernels of 256..2048 need a few registers above 128: held to 128 they
// spill one to three words per lane and keep four waves per SIMD, which
// measured 4% faster than three waves without a spill.
template <int MODE, int THREADS, int LDS_BYTES, int WPE, int ANY, class... Ss>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_trip(const CavDesc* __restrict__ descs,
                                                  const int4* __restrict__ tasks, int ntasks,
                                                  unsigned* __restrict__ ctrl, int chunk) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[LDS_BYTES];
    __shared__ double red[4 * 16];
    __shared__ int s_ticket;
    __shared__ int s_ok;
    unsigned* head = ctrl + CTRL_HEAD;
    unsigned* done = ctrl + CTRL_ROWDONE;
    for (;;) {
        if (threadIdx.x == 0)
            s_ticket = (int)__hip_atomic_fetch_add(head, (unsigned)chunk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int t0 = __builtin_amdgcn_readfirstlane(s_ticket);
        if (t0 >= ntasks) break;
        const int t1 = t0 + chunk < ntasks ? t0 + chunk : ntasks;
        for (int t = t0; t < t1; ++t) {
            const int4 tk = tasks[t];
            const int cav = __builtin_amdgcn_readfirstlane(tk.x);
            const int kind = __builtin_amdgcn_readfirstlane(tk.y);
            const int blk = __builtin_amdgcn_readfirstlane(tk.z);
            const CavDesc& d = descs[cav];
            bool run = true;
            if (kind == TASK_COL) {
                if (threadIdx.x == 0) {
                    // bounded wait: a dependency that never completes (a bad task
                    // table) marks the cavity failed and releases its waiters
                    const unsigned need = (unsigned)d.nrb + ctrl[CTRL_EXTRA];
                    const unsigned limit = ctrl[CTRL_SPIN] ? ctrl[CTRL_SPIN] : (1u << 25);   // ~2 s
                    unsigned spins = 0;
                    // relaxed polls; the acquire fence after the loop pairs
                    // with the row tasks' release increments (an acquire on
                    // every poll would invalidate this XCD's L2 under the
                    // row tasks still running on it)
                    while (__hip_atomic_load(done + cav, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                        if (__hip_atomic_load(ctrl + CTRL_ABORT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                        __builtin_amdgcn_s_sleep(2);
                        if (++spins > limit) {
                            (void)__hip_atomic_exchange(ctrl + CTRL_ABORT, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            break;
                        }
                    }
                    // whichever way the wait ended, a cavity whose row pass is
                    // incomplete is reported failed and its column task skipped
                    const bool ok = __hip_atomic_load(done + cav, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
                    if (!ok) d.counters[CNT_HANG] = 1u;
                    s_ok = ok ? 1 : 0;
                }
                // one acquire suffices: it invalidates this CU's L1 and this
                // XCD's L2, which every wave of the workgroup reads through
                if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __syncthreads();
                run = __builtin_amdgcn_readfirstlane(s_ok) != 0;
                // the trip's sums, folded once per trip (sheet 0 only)
                if (run && blk == 0 && threadIdx.x < 64 && d.trace) finalize_sums(d);
            }
            if (run) (run_if<MODE, ANY, Ss>(d, kind, blk, smem, red) || ...);
            if (kind == TASK_ROW) {
                // each wave waits for its stores to reach L2; after the
                // barrier one device-scope release writes the XCD's L2 back
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                __syncthreads();
                if (threadIdx.x == 0)
                    __hip_atomic_fetch_add(done + cav, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        const unsigned old = __hip_atomic_fetch_add(ctrl + CTRL_EXIT, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (old == gridDim.x - 1) {
            // counters change only by atomic read-modify-writes, resets included
            const int ncav = (int)ctrl[CTRL_NCAV];
            for (int c = 0; c < ncav; ++c) atomic_zero(done + c);
            atomic_zero(ctrl + CTRL_HEAD);
            atomic_zero(ctrl + CTRL_ABORT);
            atomic_zero(ctrl + CTRL_EXIT);
        }
    }
}

// Grouped launch: one workgroup per task of one pass (all row blocks, or
// all column blocks, of every cavity); the kernel boundary orders the passes.
// Consecutive workgroups are dealt round-robin to the eight XCDs.  Column
// tasks are renumbered so that each XCD walks one contiguous run of the task
// list instead: a column block reads one tile per row block, strided across
// the field, and neighbouring blocks then share their rows' DRAM pages and
// the XCD's L2 (about 5% off the column pass at 64 x 1024^2; the row pass,
// whose tasks each stream one contiguous span, gains nothing and keeps the
// launch order).
// Column tasks of single-size groups bring the cavity's propagator table hx
// into LDS together with their tile, so the propagator multiply in the middle
// of the transforms reads LDS instead of waiting on global loads.
template <int ANY, class S>
__device__ __forceinline__ void col_task_hx_lds(const CavDesc& d, int cb, unsigned char* smem) {
    cx<float>* lds = reinterpret_cast<cx<float>*>(smem);
    if constexpr (takes_trans<ANY>()) {
        if (d.prop_kind == 2) {
            col_task<S, float, COL_PROP, PROP_TRANS>(d, cb, lds);
            return;
        }
    }
    ColRegs<S, float, true> in;
    col_load<S, float, COL_PROP, true>(d, cb, in);
    col_body<S, float, COL_PROP, PROP_TABLE, TW_GLOBAL, true>(d, cb, lds, in, [] {}, nullptr,
                                                               lds + S::LDS_ELEMS);
}

template <int MODE, int KIND, int THREADS, int LDS_BYTES, int WPE, int ANY, class... Ss>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_pass(
    const CavDesc* __restrict__ descs, const int4* __restrict__ tasks) {
    constexpr bool HXLDS = sizeof...(Ss) == 1 && KIND == TASK_COL &&
                           LDS_BYTES + ((HXN<Ss, float> * 8) + ... + 0) + 4 * 16 * 8 <= 160 * 1024;
    __shared__ __attribute__((aligned(16))) unsigned char smem[LDS_BYTES + (HXLDS ? ((HXN<Ss, float> * 8) + ...) : 0)];
    __shared__ double red[4 * 16];
    unsigned t = blockIdx.x;
    if constexpr (KIND == TASK_COL) {
        // bijection of [0, G): XCD x = t % 8 gets tasks [x q + min(x, r), ...)
        const unsigned G = gridDim.x, q = G / 8u, r = G % 8u, x = t % 8u;
        t = x * q + (x < r ? x : r) + t / 8u;
    }
    const int4 tk = tasks[t];
    const int cav = __builtin_amdgcn_readfirstlane(tk.x);
    const int blk = __builtin_amdgcn_readfirstlane(tk.z);
    const CavDesc& d = descs[cav];
    if constexpr (KIND == TASK_COL) {
        // the trip's sums, folded once per trip (the descriptors of the other
        // gain sheets carry no trace)
        if (blk == 0 && threadIdx.x < 64 && d.trace) finalize_sums(d);
    }
    if constexpr (HXLDS) (col_task_hx_lds<ANY, Ss>(d, blk, smem), ...);
    else (run_if<MODE, ANY, Ss>(d, KIND, blk, smem, red) || ...);
}

// Software-pipelined grouped pass for a single grid size: a resident grid
// walks the pass's tasks with a static stride (tasks of one pass are
// independent) and issues the global loads of its next task as soon as the
// current task's tile is in LDS, so HBM traffic overlaps the FFT work.  The
// body must then issue no global load it waits for (a wait would also wait
// for the prefetch): twiddles live in LDS for the whole kernel, and the
// column pass's propagator table travels with the prefetched tile.
template <class S>
constexpr int pipe_lds_bytes(int kind) {
    return S::LDS_ELEMS * 8 + S::TW_TOTAL * 8 + (kind == TASK_COL ? HXN<S, float> * 8 : 0);
}

template <int MODE, int KIND, int THREADS, int WPE, class S>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_pass_pipe(
    const CavDesc* __restrict__ descs, const int4* __restrict__ tasks, int ntasks) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[pipe_lds_bytes<S>(KIND)];
    __shared__ double red[4 * 16];
    cx<float>* lds = reinterpret_cast<cx<float>*>(smem);
    cx<float>* ltw = lds + S::LDS_ELEMS;
    cx<float>* lhx = ltw + S::TW_TOTAL;
    int t = blockIdx.x;
    if (t >= ntasks) return;
    int cav = __builtin_amdgcn_readfirstlane(tasks[t].x);
    int blk = __builtin_amdgcn_readfirstlane(tasks[t].z);
    // every cavity of the group has the same N and precision: same twiddles
    twiddles_to_lds<S, float>(static_cast<const cx<float>*>(descs[cav].tw), ltw, opaque_tid());
    if constexpr (KIND == TASK_ROW) {
        RowRegs<S, float> in;
        row_load<S, float, MODE>(descs[cav], blk, in);
        for (;;) {
            const int tn = t + (int)gridDim.x;
            const bool more = tn < ntasks;
            const int cavn = more ? __builtin_amdgcn_readfirstlane(tasks[tn].x) : 0;
            const int blkn = more ? __builtin_amdgcn_readfirstlane(tasks[tn].z) : 0;
            row_body<S, float, MODE, TW_LDS>(descs[cav], blk, lds, red, in, [&] {
                if (more) row_load<S, float, MODE>(descs[cavn], blkn, in);
            }, ltw);
            if (!more) break;
            t = tn;
            cav = cavn;
            blk = blkn;
            __syncthreads();
        }
    } else {
        ColRegs<S, float, true> in;
        col_load<S, float, COL_PROP, true>(descs[cav], blk, in);
        for (;;) {
            const int tn = t + (int)gridDim.x;
            const bool more = tn < ntasks;
            const int cavn = more ? __builtin_amdgcn_readfirstlane(tasks[tn].x) : 0;
            const int blkn = more ? __builtin_amdgcn_readfirstlane(tasks[tn].z) : 0;
            const CavDesc& d = descs[cav];
            if (blk == 0 && threadIdx.x < 64 && d.trace) finalize_sums(d);
            col_body<S, float, COL_PROP, PROP_TABLE, TW_LDS, true>(d, blk, lds, in, [&] {
                if (more) col_load<S, float, COL_PROP, true>(descs[cavn], blkn, in);
            }, ltw, lhx);
            if (!more) break;
            t = tn;
            cav = cavn;
            blk = blkn;
            __syncthreads();
        }
    }
}

template <class... Ss>
constexpr bool pipe_fits() {
    if constexpr (sizeof...(Ss) == 1)
        return ((pipe_lds_bytes<Ss>(TASK_COL) + 4 * 16 * 8 <= 160 * 1024) && ...);
    else
        return false;
}

#define LSR_LAUNCH(KERN, G, B, ST, EV, ...)                                                  \
    do {                                                                                    \
        if ((EV).start || (EV).stop)                                                        \
            hipExtLaunchKernelGGL(KERN, G, B, 0, ST, (EV).start, (EV).stop, 0, __VA_ARGS__); \
        else                                                                                \
            hipLaunchKernelGGL(KERN, G, B, 0, ST, __VA_ARGS__);                             \
    } while (0)

// ANY = 1: kernels that run each cavity's own local-step model (groups for
// batches holding other models than the default; no pipelined form).
template <int WPE, int ANY, class... Ss>
struct GroupKernelsT {
    static constexpr int THREADS = Group<Ss...>::THREADS;
    static constexpr int LDS = Group<Ss...>::maxl();
    // the pipelined pass exists for single-size groups whose LDS (lines,
    // twiddles, propagator table) fits one workgroup
    static constexpr bool PIPE = !ANY && pipe_fits<Ss...>();

    static int launch(int mode, int grid, hipStream_t st, const CavDesc* descs, const int4* tasks,
                      int ntasks, unsigned* ctrl, int chunk, LaunchEvents ev) {
        const dim3 g(grid), b(THREADS);
        switch (mode) {
        case ROW_FIRST: LSR_LAUNCH((k_trip<ROW_FIRST, THREADS, LDS, WPE, ANY, Ss...>), g, b, st, ev, descs, tasks, ntasks, ctrl, chunk); break;
        case ROW_MID:   LSR_LAUNCH((k_trip<ROW_MID, THREADS, LDS, WPE, ANY, Ss...>), g, b, st, ev, descs, tasks, ntasks, ctrl, chunk); break;
        case ROW_LAST:  LSR_LAUNCH((k_trip<ROW_LAST, THREADS, LDS, WPE, ANY, Ss...>), g, b, st, ev, descs, tasks, ntasks, ctrl, chunk); break;
        default: return -1;
        }
        return hipGetLastError() == hipSuccess ? 0 : -3;
    }
    static int occupancy() {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_trip<ROW_MID, THREADS, LDS, WPE, ANY, Ss...>, THREADS, 0) != hipSuccess)
            return 1;
        return n > 0 ? n : 1;
    }
    // grouped launch of one pass: grid = number of tasks of that pass
    static int launch_pass(int mode, int kind, hipStream_t st, const CavDesc* descs, const int4* tasks,
                           int ntasks, LaunchEvents ev) {
        const dim3 g(ntasks), b(THREADS);
        if (kind == TASK_COL) {
            LSR_LAUNCH((k_pass<ROW_MID, TASK_COL, THREADS, LDS, WPE, ANY, Ss...>), g, b, st, ev, descs, tasks);
        } else {
            switch (mode) {
            case ROW_FIRST: LSR_LAUNCH((k_pass<ROW_FIRST, TASK_ROW, THREADS, LDS, WPE, ANY, Ss...>), g, b, st, ev, descs, tasks); break;
            case ROW_MID:   LSR_LAUNCH((k_pass<ROW_MID, TASK_ROW, THREADS, LDS, WPE, ANY, Ss...>), g, b, st, ev, descs, tasks); break;
            case ROW_LAST:  LSR_LAUNCH((k_pass<ROW_LAST, TASK_ROW, THREADS, LDS, WPE, ANY, Ss...>), g, b, st, ev, descs, tasks); break;
            default: return -1;
            }
        }
        return hipGetLastError() == hipSuccess ? 0 : -3;
    }
    // pipelined pass (single-size groups): resident grid of `grid` workgroups
    static int launch_pipe(int mode, int kind, hipStream_t st, const CavDesc* descs, const int4* tasks,
                           int ntasks, int grid, LaunchEvents ev) {
        if constexpr (PIPE) {
            const dim3 g(grid < ntasks ? grid : ntasks), b(THREADS);
            if (kind == TASK_COL) {
                LSR_LAUNCH((k_pass_pipe<ROW_MID, TASK_COL, THREADS, WPE, Ss...>), g, b, st, ev, descs, tasks, ntasks);
            } else {
                switch (mode) {
                case ROW_FIRST: LSR_LAUNCH((k_pass_pipe<ROW_FIRST, TASK_ROW, THREADS, WPE, Ss...>), g, b, st, ev, descs, tasks, ntasks); break;
                case ROW_MID:   LSR_LAUNCH((k_pass_pipe<ROW_MID, TASK_ROW, THREADS, WPE, Ss...>), g, b, st, ev, descs, tasks, ntasks); break;
                case ROW_LAST:  LSR_LAUNCH((k_pass_pipe<ROW_LAST, TASK_ROW, THREADS, WPE, Ss...>), g, b, st, ev, descs, tasks, ntasks); break;
                default: return -1;
                }
            }
            return hipGetLastError() == hipSuccess ? 0 : -3;
        } else {
            (void)mode; (void)kind; (void)st; (void)descs; (void)tasks; (void)ntasks; (void)grid; (void)ev;
            return -1;
        }
    }
    // resident workgroups per CU of the pipelined row (kind 0) / column pass
    static int occupancy_pipe(int kind) {
        if constexpr (PIPE) {
            int n = 0;
            hipError_t e = kind == TASK_COL
                ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_pass_pipe<ROW_MID, TASK_COL, THREADS, WPE, Ss...>, THREADS, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_pass_pipe<ROW_MID, TASK_ROW, THREADS, WPE, Ss...>, THREADS, 0);
            return (e == hipSuccess && n > 0) ? n : 1;
        } else {
            (void)kind;
            return 0;
        }
    }
    static KernelVariant variant() {
        KernelVariant v{&launch, &launch_pass, &occupancy, WPE, nullptr, nullptr};
        if constexpr (PIPE) {
            v.launch_pipe = &launch_pipe;
            v.occupancy_pipe = &occupancy_pipe;
        }
        return v;
    }
};

template <int WPE, class... Ss>
using GroupKernels = GroupKernelsT<WPE, 0, Ss...>;

template <class... Ss>
GroupInfo group_info(std::initializer_list<KernelVariant> vars, int alt = 0, int any_model = 0) {
    GroupInfo gi{};
    gi.threads = Group<Ss...>::THREADS;
    gi.alt = alt;
    gi.any_model = any_model;
    gi.nsizes = 0;
    ((gi.shapes[gi.nsizes] = shape_info<Ss>(), gi.sizes[gi.nsizes++] = Ss::N), ...);
    gi.nvariants = 0;
    for (const KernelVariant& v : vars) gi.var[gi.nvariants++] = v;
    return gi;
}

}  // namespace lsr
