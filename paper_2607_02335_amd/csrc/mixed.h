// Launches that mix problems of different degrees.
//
// A batched launch of one kernel covers the problems of one degree.  A mixed
// launch covers the problems of the degrees 7, 3 and 2 together in one
// kernel: the work of each degree is a list of items (the workgroups of that
// degree's own kernel over its problems' tiles), the lists of the degrees
// follow each other in one grid, and every workgroup runs one item of one
// degree (degree-uniform workgroups).  The bodies are the single-degree
// kernels' own code, called with the item as the workgroup index and the
// item count as the grid, so every problem's result is the same bit for bit
// whichever way it is launched.  Segments are ordered heaviest degree first,
// so the long items start early; segment offsets are multiples of 8, so item
// i runs on XCD i % 8 as in a launch of the body's own kernel.  A workgroup
// runs exactly one item: a loop over items (a persistent grid) would let the
// compiler keep one body's loop-invariant values live in registers across
// the whole launch, which measured 67 -> 127 VGPRs for the FP32 solves.
#pragma once

#include <vector>

#include "fem_internal.h"
#include "launch.h"

namespace fem {

constexpr int kMixSegs = 3;
// segment k of a mixed launch holds the problems of degree mix_degree(k)
__host__ __device__ constexpr int mix_degree(int k) { return k == 0 ? 7 : k == 1 ? 3 : 2; }
inline bool mix_has_degree(int p) { return p == 7 || p == 3 || p == 2; }

struct MixSeg {
    LaunchTable L;   // the segment's problems: device table, tile ranges of its body
    int count;       // items of the segment (a multiple of 8)
    int wg_begin;    // workgroup of its first item (a multiple of 8)
};

struct MixTable {
    MixSeg seg[kMixSegs];
};

struct NoArg {};

constexpr int lds_max(int a, int b) { return a > b ? a : b; }

// A body B provides: Arg (its by-value kernel argument), kLds (bytes of
// LDS), and run(L, arg, item, items, smem) doing what workgroup `item` of a
// grid of `items` workgroups of its own kernel does.
template <class B, class A>
__device__ __forceinline__ void mix_segment(const MixSeg& g, const A& a, char* smem) {
    B::run(g.L, a, (int)blockIdx.x - g.wg_begin, g.count, smem);
}

template <class B0, class B1, class B2>
__global__ void __launch_bounds__(256)
k_mixed(MixTable T, typename B0::Arg a0, typename B1::Arg a1, typename B2::Arg a2) {
    constexpr int kL = lds_max(16, lds_max(B0::kLds, lds_max(B1::kLds, B2::kLds)));
    __shared__ __align__(16) char smem[kL];
    if ((int)blockIdx.x < T.seg[1].wg_begin) mix_segment<B0>(T.seg[0], a0, smem);
    else if ((int)blockIdx.x < T.seg[2].wg_begin) mix_segment<B1>(T.seg[1], a1, smem);
    else mix_segment<B2>(T.seg[2], a2, smem);
}

// Host side.  Splits `ents` (every degree in the mixed set) into the
// segments, keeping their order within a degree; tiles(p, e) is problem e's
// tile count in the degree-p body, items(p, t) the items (workgroups of the
// body's own grid) covering t tiles.  All entries go up in one table.
template <class TilesF, class ItemsF>
hipError_t mix_build(const ProbEntry* ents, int nprob, TableStager* st, hipStream_t s, TilesF&& tiles,
                     ItemsF&& items, MixTable& T, int& grid) {
    if (!st) return hipErrorInvalidValue;
    std::vector<ProbEntry> v;
    v.reserve(nprob);
    int off[kMixSegs];
    for (int k = 0; k < kMixSegs; ++k) {
        const int p = mix_degree(k);
        off[k] = (int)v.size();
        int t = 0;
        for (int i = 0; i < nprob; ++i) {
            if (ents[i].p != p) continue;
            ProbEntry e = ents[i];
            e.tile_begin = t;
            e.ntiles = tiles(p, e);
            t += e.ntiles;
            v.push_back(e);
        }
        T.seg[k].L = LaunchTable{};
        T.seg[k].L.nprob = (int)v.size() - off[k];
        T.seg[k].L.total_tiles = t;
    }
    if ((int)v.size() != nprob) return hipErrorInvalidValue;
    const ProbEntry* dev = nullptr;
    hipError_t err = st->upload(v.data(), nprob, s, &dev);
    if (err != hipSuccess) return err;
    long b = 0;
    for (int k = 0; k < kMixSegs; ++k) {
        MixSeg& g = T.seg[k];
        g.L.tab = dev + off[k];
        const int c = (g.L.nprob > 0 && g.L.total_tiles > 0) ? items(mix_degree(k), g.L.total_tiles) : 0;
        g.count = (c + 7) / 8 * 8;
        g.wg_begin = (int)b;
        b += g.count;
    }
    if (b > 0x7fffffffL) return hipErrorInvalidValue;
    grid = (int)b;
    return hipSuccess;
}

// Number of distinct degrees of the mixed set among `ents`, or -1 if some
// entry has a degree outside it.
inline int mix_degrees(const ProbEntry* ents, int nprob) {
    bool seen[kMaxP + 1] = {};
    for (int i = 0; i < nprob; ++i) {
        if (!mix_has_degree(ents[i].p)) return -1;
        seen[ents[i].p] = true;
    }
    return (int)seen[2] + (int)seen[3] + (int)seen[7];
}

}  // namespace fem
