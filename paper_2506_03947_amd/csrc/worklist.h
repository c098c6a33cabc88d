// Work-list dispatch for batched launches: a launch covers the members of a list
// (independent problems), member q owning nb(q) consecutive virtual blocks; members
// whose live flag is clear own none.  The first wave of every workgroup scans the live
// members' block counts into LDS (at most kListMax members), then the workgroup walks
// virtual blocks blockIdx.x, blockIdx.x + gridDim.x, ... below the live total.  The
// grid is sized for the whole list, but converged members cost nothing beyond the scan.
//
// Each member's first virtual block is rounded up to a multiple of 8 and the grid is a
// multiple of 8, so a virtual block keeps the XCD of its workgroup (workgroups are
// dealt round-robin to the 8 XCDs) and the member's local block index has the same
// residue mod 8: the XCD-aware tile orders of the kernels stay intact.  A local
// index past the member's own count (padding) does no work.
#pragma once

#include <hip/hip_runtime.h>

namespace ac {

constexpr int kListMax = 256;      // members per list
constexpr int kListWaves = 8192;   // waves of the largest work-list grid (256 CUs x 32)

// Grid of a work-list launch of `wpb` waves per workgroup over members whose block
// counts sum to `blocks`: every virtual block when all members are live, but no more
// workgroups than about two rounds of residency, so that a list whose members have
// mostly converged costs one short scan per workgroup.
inline int list_grid(long long blocks, int members, int wpb) {
    long long g = blocks + 7LL * members;
    g = (g + 7) / 8 * 8;
    const long long cap = kListWaves / (wpb < 1 ? 1 : wpb) / 8 * 8;
    if (g > cap) g = cap;
    return g < 8 ? 8 : static_cast<int>(g);
}

struct LiveBlocks {
    int n, total;
};

__device__ __forceinline__ int wave_incl_scan(int x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// LDS copy of the scan: first virtual block and own block count of every member
struct ListLds {
    int excl[kListMax];
    int nb[kListMax];
    int total;
};

__device__ __forceinline__ ListLds& list_lds() {
    __shared__ ListLds L;
    return L;
}

// nbf(q): block count of member q;  livef(q): whether it computes.  Every thread of the
// workgroup calls this once, before any divergent exit (it holds a barrier).
template <typename NbF, typename LiveF>
__device__ __forceinline__ LiveBlocks live_blocks(int n, NbF nbf, LiveF livef) {
    ListLds& S = list_lds();
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        int carry = 0;
        for (int c = 0; c * 64 < n; ++c) {
            const int q = c * 64 + lane;
            int nb = 0, pad = 0;
            if (q < n) {
                nb = nbf(q);
                pad = livef(q) ? (nb + 7) & ~7 : 0;
            }
            const int incl = wave_incl_scan(pad);
            S.excl[q] = q < n ? carry + incl - pad : 0x7fffffff;
            S.nb[q] = nb;
            carry += __shfl(incl, 63, 64);
        }
        if (lane == 0) S.total = carry;
    }
    __syncthreads();
    return LiveBlocks{n, S.total};
}

// Member, local block and the member's block count of virtual block v < W.total
// (uniform across the wave); false for a padding block.
__device__ __forceinline__ bool live_block(const LiveBlocks& W, int v, int& q, int& local, int& nb) {
    const ListLds& S = list_lds();
    const int lane = threadIdx.x & 63;
    int k = 0;
    for (int c = 0; c * 64 < W.n; ++c) k += __popcll(__ballot(S.excl[c * 64 + lane] <= v));
    q = __builtin_amdgcn_readfirstlane(k - 1);  // the last member starting at or before v
    nb = __builtin_amdgcn_readfirstlane(S.nb[q]);
    local = __builtin_amdgcn_readfirstlane(v - S.excl[q]);
    return local < nb;
}

// Member q's argument record of a work list, read through the constant address space:
// the records do not change during a launch, so the compiler may fetch them with
// scalar loads even inside the loop over virtual blocks.
template <typename T>
__device__ __forceinline__ const T& list_args(const void* args, int q) {
    typedef const T __attribute__((address_space(4))) CT;
    CT* p = (CT*)(reinterpret_cast<unsigned long long>(args)) + q;
    return *(const T*)p;
}

}  // namespace ac
