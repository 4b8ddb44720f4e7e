// so_batch.h -- persistent form of the fused pair kernel for batches of
// problems (several walker sets, shadow sets and orbital counts in one call).
//
// A launch serves up to SO_JOBS_PER_LAUNCH problems of one kernel class
// (same MFMA tile count T, same ne = n - eta and same formation precision).  Their work items
// (walker, range of shadows) are numbered problem by problem, the problem
// with the costliest items first (longest-processing-time order), walkers
// fastest within a shadow range so that concurrent waves share C'_s in L2.
// Every wave takes the next item from a counter in global memory until the
// items run out, so the grid is sized to the machine rather than to the
// problem, and each wave ends after its last item.
#pragma once
#include "so_common.h"
#include "so_pair.h"

#define SO_JOBS_PER_LAUNCH 2

struct PairJob {
    const void *Xa, *Ca;   // formation operands (FP64 or single precision)
    double2 *pairs;
    so_u64 *fb_count;
    int64_t *fb_list;
    int32_t *wstat;
    int64_t fb_cap, S, item0, nitems;
    int n, eta, W, spw;
};
struct PairJobs {
    PairJob job[SO_JOBS_PER_LAUNCH];
    RedTab tab[SO_JOBS_PER_LAUNCH];
    int njobs;
    int64_t total;
};

// counter[0] = 0 (a kernel rather than a memset: the sequence may be captured
// into a graph)
__global__ void k_zero_u32(uint32_t *counter) {
    if (threadIdx.x == 0) counter[0] = 0u;
}

template <int T, int NE, bool MIX>
__global__ __launch_bounds__(64, 2) void k_pair_persistent(PairJobs J, uint32_t *__restrict__ counter) {
    for (;;) {
        uint32_t it = 0u;
        if (threadIdx.x == 0) it = atomicAdd(counter, 1u);
        it = (uint32_t)__shfl((int)it, 0, 64);
        if ((int64_t)it >= J.total) break;
        const int p = (J.njobs > 1 && (int64_t)it >= J.job[1].item0) ? 1 : 0;
        const PairJob &jb = (p == 0) ? J.job[0] : J.job[1];
        const RedTab &tb = (p == 0) ? J.tab[0] : J.tab[1];
        const int64_t local = (int64_t)it - jb.item0;
        const int64_t y = local / jb.W;
        const int w = (int)(local - y * jb.W);
        const int64_t sb0 = y * jb.spw;
        const int64_t sb1 = min(jb.S, sb0 + jb.spw);
        pair_range<T, NE, MIX>(jb.n, jb.eta, jb.Xa, jb.Ca, jb.S, tb, jb.pairs, jb.fb_count, jb.fb_list, jb.fb_cap,
                          jb.wstat, w, sb0, sb1);
    }
}
