// so_batch.h -- one fused launch of the pair kernel over a batch of problems
// (several walker sets, shadow sets and orbital counts).
//
// Every fused problem of the batch, whatever its kernel class (MFMA tile
// count T, ne = n - eta), is served by the same launch: the kernel holds the
// per-class code paths (compile-time instances of pair_range, grouped in
// register levels) and dispatches on the class of its work item.
//
// Work items are (walker, range of spw shadows), one per workgroup.  MI355X
// dispatches workgroup b to XCD b mod 8, and the workgroups of XCD x take the
// items of the walkers w = x (mod 8) of every problem, so each XCD keeps its
// own eighth of the walker matrices hot in its L2 and streams each shadow's
// covariance once.  The items of an XCD form a sequence of rounds: round r
// holds the next per_round[p] items of each problem p (costliest problem
// first), so with R rounds every problem progresses at the same relative
// rate, and with R = 1 the order is longest-processing-time, problem by
// problem.  Within a problem items run walkers fastest, so the concurrent
// workgroups of an XCD share the covariances of a shadow range.  The
// hardware dispatcher hands out the workgroups in order as compute units free
// up, which balances the load without a software queue: a persistent loop
// over an atomic queue was measured slower, since its loop-carried state
// pushes the class paths into register spills.
#pragma once
#include "so_common.h"
#include "so_pair.h"

#define SO_BATCH_XCD 8
#define SO_BATCH_MAXJOBS 16

// One problem of a batch launch, written to device memory by k_batch_setup.
struct BatchJob {
    const void *Xa, *Ca;   // formation operands (FP64 or single precision)
    double2 *pairs;
    so_u64 *fb_count;
    int64_t *fb_list;
    int32_t *wstat;
    int64_t fb_cap, S;
    int64_t len[SO_BATCH_XCD];         // items of XCD x: Wx * nY
    int64_t per_round[SO_BATCH_XCD];   // items of XCD x per round
    int n, eta, W, spw, cls;           // cls = 16 T + ne
    int pad_;
    RedTab tab;
};
struct BatchHdr {
    int64_t round_len[SO_BATCH_XCD];   // sum over problems of per_round[x]
    int64_t qlen[SO_BATCH_XCD];        // positions of XCD x: rounds * round_len[x]
    int njobs;
    int pad_;
};

// job and header writers (kernels rather than copies: the sequence may be
// captured into a graph)
__global__ void k_batch_setup(BatchJob job, BatchJob *__restrict__ dst) {
    const int t = threadIdx.x;
    // copy the job word by word (uniform work, one wave)
    const uint32_t *src = reinterpret_cast<const uint32_t *>(&job);
    uint32_t *d = reinterpret_cast<uint32_t *>(dst);
    for (int i = t; i < (int)(sizeof(BatchJob) / 4); i += 64) d[i] = src[i];
}
__global__ void k_batch_header(BatchHdr hdr, BatchHdr *__restrict__ dst) {
    const int t = threadIdx.x;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(&hdr);
    uint32_t *d = reinterpret_cast<uint32_t *>(dst);
    for (int i = t; i < (int)(sizeof(BatchHdr) / 4); i += 64) d[i] = src[i];
}

// the class-specific body of one item
template <int LEVEL, bool MIX>
__device__ __forceinline__ void batch_item(const BatchJob &jb, int w, int64_t sb0, int64_t sb1) {
#define SO_BCASE(TT, NN)                                                                                       \
    case 16 * TT + NN:                                                                                         \
        if constexpr (pair_class_level(TT, NN, MIX) <= LEVEL)                                                \
            pair_range<TT, NN, MIX, false, true>(jb.n, jb.eta, jb.Xa, jb.Ca, jb.S, jb.tab, jb.pairs, jb.fb_count, jb.fb_list, \
                                    jb.fb_cap, jb.wstat, w, sb0, sb1);                                         \
        break;
#define SO_BFULL(TT, NN)                                                                                       \
    case 256 + 16 * TT + NN:                                                                                   \
        if constexpr (pair_class_level(TT, NN, MIX) <= LEVEL)                                                \
            pair_range<TT, NN, MIX, true, true>(jb.n, jb.eta, jb.Xa, jb.Ca, jb.S, jb.tab, jb.pairs, jb.fb_count, jb.fb_list, \
                                    jb.fb_cap, jb.wstat, w, sb0, sb1);                                         \
        break;
    switch (jb.cls) {
        SO_BFULL(1, 2) SO_BFULL(1, 4) SO_BFULL(1, 6) SO_BFULL(2, 8) SO_BFULL(3, 10) SO_BFULL(3, 12)
        SO_BCASE(1, 2) SO_BCASE(1, 4) SO_BCASE(1, 6) SO_BCASE(1, 8)
        SO_BCASE(2, 2) SO_BCASE(2, 4) SO_BCASE(2, 6) SO_BCASE(2, 8) SO_BCASE(2, 10) SO_BCASE(2, 12)
        SO_BCASE(3, 2) SO_BCASE(3, 4) SO_BCASE(3, 6) SO_BCASE(3, 8) SO_BCASE(3, 10) SO_BCASE(3, 12)
        default: break;
    }
#undef SO_BCASE
#undef SO_BFULL
}

// grid 8 max_x qlen[x], one wave per block
template <int LEVEL, bool MIX>
__global__ __launch_bounds__(64, LEVEL == 0 ? 3 : 2) void k_pair_batch(const BatchJob *__restrict__ jobs,
                                                      const BatchHdr *__restrict__ hdr) {
    const int x = blockIdx.x & (SO_BATCH_XCD - 1);
    const int64_t pos = (int64_t)(blockIdx.x / SO_BATCH_XCD);
    if (pos >= hdr->qlen[x]) return;
    const int njobs = hdr->njobs;
    const int64_t rl = hdr->round_len[x];
    const int64_t r = pos / rl;
    int64_t o = pos - r * rl;
    int p = 0;
    while (p < njobs - 1 && o >= jobs[p].per_round[x]) {
        o -= jobs[p].per_round[x];
        ++p;
    }
    const BatchJob &jb = jobs[p];
    const int64_t i = r * jb.per_round[x] + o;
    if (i >= jb.len[x]) return;   // this problem has run out in XCD x's sequence
    const int Wx = (jb.W - x + SO_BATCH_XCD - 1) / SO_BATCH_XCD;   // walkers w = x (mod 8)
    const int64_t y = i / Wx;
    const int w = (int)(i - y * Wx) * SO_BATCH_XCD + x;
    const int64_t sb0 = y * jb.spw;
    const int64_t sb1 = min(jb.S, sb0 + jb.spw);
    batch_item<LEVEL, MIX>(jb, w, sb0, sb1);
}
