// Load balancing of per-point candidate walks over the lanes of a wavefront.
//
// The distance queries test each point against a short list of candidates
// (the segments or disks its grid cell lists).  Walked one point per lane, a
// wavefront takes as many dependent gather-and-test steps as its longest
// list.  Instead, each round lines up the remaining candidates of the
// wavefront's points in lane order and gives position t of that sequence to
// lane t: the lane tests the candidate against its owner's point.  A
// wavefront then takes about (candidates in total) / 64 rounds.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprim/warp/warp_scan.hpp>
#include <stdint.h>

namespace spade {

// One round: this lane's point has rem candidates left, of which c (at most
// 64, so that the prefix sums stay small) take the positions [pre, incl)
// of the round's sequence (a wavefront scan, rocPRIM's cross-lane warp scan);
// positions below ntake (at most 64) are tested.
// Lane t tests position t, which belongs to lane o (the first lane whose
// inclusive prefix exceeds t, found by a binary search over the lanes) and
// is the (t - opre)-th of o's candidates this round.
struct WaveRound {
    uint32_t c, pre, incl, ntake, opre;
    int o;
};

// Called by every lane of the wavefront.
__device__ __forceinline__ WaveRound wave_round(uint32_t rem, int lane)
{
    WaveRound w;
    w.c = min(rem, 64u);
    uint32_t incl, total;
    typename rocprim::warp_scan<uint32_t, 64>::storage_type scan_storage;
    rocprim::warp_scan<uint32_t, 64>().inclusive_scan(w.c, incl, total, scan_storage, rocprim::plus<uint32_t>());
    w.incl = incl;
    w.pre = incl - w.c;
    w.ntake = min(total, 64u);
    int o = 0;
    for (int st = 32; st > 0; st >>= 1)
        if (__shfl(incl, o + st - 1, 64) <= (uint32_t)lane) o += st;
    w.o = o;
    w.opre = __shfl(w.pre, o, 64);
    return w;
}

// The number of this lane's candidates tested in the round, and their
// positions as a lane mask.
__device__ __forceinline__ uint32_t wave_round_len(const WaveRound &w)
{
    return (w.c != 0u && w.pre < 64u) ? min(w.incl, 64u) - w.pre : 0u;
}

__device__ __forceinline__ unsigned long long wave_round_mask(const WaveRound &w)
{
    const uint32_t len = wave_round_len(w);
    return len == 0u ? 0ull : ((len >= 64u ? ~0ull : ((1ull << len) - 1ull)) << w.pre);
}

// Positions of the same owner before this lane's in the round (0 for lanes
// past ntake).
__device__ __forceinline__ unsigned long long wave_round_before(const WaveRound &w, int lane)
{
    return (uint32_t)lane < w.ntake ? (((1ull << lane) - 1ull) & ~((1ull << w.opre) - 1ull)) : 0ull;
}

}  // namespace spade
