// Key table of the greedy policy, shared by the Picard walk and the serial sweep.
//
// key[b][r][w] = (pos << S) | w, where pos is the position of warehouse w in region r's
// increasing (cost[b][w][r], w) order: 16-bit keys with S = 8 when N <= 255, else 32-bit
// keys with S = 16.  (At N = 256 the key of warehouse 255 in last place would be 0xffff,
// the all-ones value that stands for "no warehouse with stock".)  The least key among warehouses with stock names the greedy choice
// (least cost, lowest index on ties).  Per trajectory the table holds R rows of npad
// keys; rows are padded to 32 bytes with all-ones keys, which are never selected.
#pragma once

#include "pk_internal.h"

namespace pk {

template <typename KeyT> __host__ __device__ inline int tab_npad(int N)
{
    constexpr int per = 32 / (int)sizeof(KeyT);
    return (N + per - 1) / per * per;
}
template <typename KeyT> __host__ __device__ inline int64_t tab_stride(int N, int R)
{
    return (int64_t)R * tab_npad<KeyT>(N);
}
template <typename KeyT> __host__ __device__ constexpr int key_shift()
{
    return sizeof(KeyT) == 2 ? 8 : 16;
}

// Preference lists (N <= 128): pref[b][r][i] = the warehouse with key position i in region
// r, i < N (the inverse of the key table's positions); rows padded to 16 bytes with 127,
// a warehouse that never has stock when N < 128 (at N = 128 there is no padding).
__host__ __device__ inline int pref_npad(int N) { return (N + 15) & ~15; }

} // namespace pk
