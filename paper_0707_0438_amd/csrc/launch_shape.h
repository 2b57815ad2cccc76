// Launch shape of the pairwise kernel: how an evaluation of n_i
// i-particles against n_j j-particles is cut into work-groups and j-ranges
// (Section 3.2's bundles and j-split), and the default shape for a size.
// Shared by the host launch code and, for block steps, by the device.
#pragma once

#include <stdint.h>

#include <algorithm>

#include "nbody.h"

namespace nb {

// Launch geometry of the pairwise kernel for an i-list of ni against nj:
// nb i-blocks of per_blk particles and S j-ranges of jchunk records (a
// multiple of the tile).  Enough work-groups to cover the 256 CUs several
// times, with at least min_tiles tiles per j-range.  Used by the host for direct
// calls and by the device for block steps whose size only it knows.  Small
// self-gravitating sets are latency-bound: a j-range of one tile per
// work-group was the fastest on MI355X from N = 256 to 4096 (N = 1024:
// pairwise 10.7 us against 28 us with four tiles per range).
__host__ __device__ inline void split_plan(int64_t ni, int64_t nj, int per_blk, int tile_j, int split_req,
                                           int* nb_out, int* S_out, int* jchunk_out, int min_tiles = 1) {
    const int64_t nb = (ni + per_blk - 1) / per_blk;
    int64_t S = split_req;
    if (S <= 0) {
        const int64_t target = 2048;
        if (nb <= 0 || nb >= target / 2) {
            S = 1;
        } else {
            S = (target + nb - 1) / nb;
            int64_t smax = nj / ((int64_t)min_tiles * tile_j);
            if (smax < 1) smax = 1;
            if (S > smax) S = smax;
            if (S < 1) S = 1;
        }
    }
    int64_t jchunk = (nj + S - 1) / S;
    jchunk = ((jchunk + tile_j - 1) / tile_j) * tile_j;
    if (jchunk <= 0) jchunk = tile_j;
    int64_t S2 = (nj + jchunk - 1) / jchunk;
    if (S2 < 1) S2 = 1;
    *nb_out = (int)nb;
    *S_out = (int)S2;
    *jchunk_out = (int)jchunk;
}

// Number of j-ranges for an i-list of ni against nj (see split_plan).  Long
// evaluations also split j: with at least kLongWG work-groups in all, the
// last, partly filled round of resident work-groups is a small part of the
// launch.  Each range keeps at least kLongTiles tiles, and the partials stay
// below (kLongWG + i-blocks) x (i per block) x 56 B.  On MI355X at N = 2^20
// this took the large DS evaluation from 749 to 726 ms (4096 i-blocks, 8
// ranges), and 2^17 i against 2^20 j from 96 to 90 ms (64 ranges).
constexpr int64_t kLongWG = 32768;
constexpr int64_t kLongTiles = 64;
// The long-evaluation split keeps its partial sums (8 rows of 8 bytes per
// i and range at most) within this many bytes.
constexpr int64_t kLongPartBytes = (int64_t)1 << 31;
inline int choose_split(int64_t ni, int64_t nj, const nbody_tile& t) {
    int nb, S, jc;
    split_plan(ni, nj, t.wg * t.ipt, t.tile_j, 0, &nb, &S, &jc);
    const int64_t per = (int64_t)t.wg * t.ipt;
    const int64_t nbl = (ni + per - 1) / per;
    int64_t Sl = nbl > 0 ? (kLongWG + nbl - 1) / nbl : 1;
    Sl = std::min<int64_t>(Sl, nj / (kLongTiles * t.tile_j));
    Sl = std::min<int64_t>(Sl, kLongPartBytes / (64 * std::max<int64_t>(ni, 1)));
    return (int)std::max<int64_t>(S, Sl);
}

// Default launch shape when neither an override nor a tuned entry exists:
// the fastest shape of the MI355X sweep at 2^20 x 2^20 (256-record LDS
// tiles, software-pipelined LDS reads; two i per lane for DS, one for plain
// FP32) for large problems,
// 64-record tiles for small ones (more j-ranges to spread over the CUs), and
// for the smallest j sets (latency-bound: the time is one work-group's
// sweep) 32- or 16-record tiles in one-wave work-groups.  short_tiles: the
// evaluation kind has those shapes.
inline nbody_tile default_tile(int prec, int64_t ni, int64_t nj, bool short_tiles = true) {
    nbody_tile t;
    const bool large = (double)ni * (double)nj >= 4294967296.0;
    t.tile_j = large ? 256 : 64;
    t.wg = large ? 256 : 128;
    if (!large && short_tiles && nj <= 2048) {
        t.tile_j = nj <= 512 ? 16 : 32;
        t.wg = 64;
    }
    // DS at large sizes: two i per lane (with the long-evaluation split,
    // 683 ms at 2^20 against 709-713 ms for one i per lane, same box);
    // plain FP32 keeps one i per lane (578-580 ms against 594)
    t.ipt = (large && prec == 1) ? 2 : 1;
    t.split = 0;
    t.jsrc = 0;
    t.unroll = large ? (prec == 1 ? 101 : 102) : 0;
    t.waves = 0;
    return t;
}

// Defaults of the force-only (kind 1) and nearest-neighbour (kind 2)
// evaluations: the fastest shapes of the MI355X sweep at 2^20 x 2^20; small
// problems take the small default shape.
inline nbody_tile default_tile_kind(int kind, int prec, int64_t ni, int64_t nj) {
    // the full evaluation's default (two i per lane for DS at large sizes) is
    // also the fastest force-only and neighbour shape of the sweeps
    return default_tile(prec, ni, nj, kind == 0);
}

}  // namespace nb
