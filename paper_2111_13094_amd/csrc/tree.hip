// tree.hip -- the spatial kD-tree on gfx950: pre-subdivision, refinement of leaves with
// many samples, copies of the parent mixture into new leaves, leaf initialisation, and
// the reordering of the samples by leaf that the batched fit consumes (Dodik et al.,
// arXiv 2111.13094, Sec. 4.2 "Refinement of the spatial kD-tree", Sec. 4.3
// "Initialization").
//
// Refinement runs in rounds. Each round: every sample is located in the current tree;
// the samples are ordered by leaf index, each leaf's samples contiguous and in index
// order (a stable LSD radix sort in the first round, a stable partition of the previous
// order after it); each leaf of the round with more than c samples gets its FP64 position
// sums, minima and maxima from one work group (fixed reduction order); one work group
// decides the splits in leaf order (a block prefix sum numbers the new nodes and leaves);
// new leaves get copies of their parent's mixture and Robbins-Monro state. The host reads
// the number of splits after each round and stops when a round makes none; the last
// round's order is the final one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "timing.hpp"

namespace sdmm {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;                      // keys per thread per block
constexpr int kSortTile = kSortThreads * kSortItems;  // keys per block
constexpr int kRadixBits = 8, kRadix = 1 << kRadixBits;
constexpr int kMaxRounds = 64;

struct TreePtrs {
    int32_t max_nodes, max_leaves;
    int32_t *counts, *axis, *left, *leaf;
    double* split;
    int32_t* leaf_node;
    double *lo, *hi;
    int32_t* init;
};

// ---------------------------------------------------------------------------------
// pre-subdivision: node n of the complete tree (children 2n + 1, 2n + 2); its path from
// the root is the binary expansion of n + 1 after the leading one (0 = left)
// ---------------------------------------------------------------------------------
__global__ void tree_init_kernel(TreePtrs t, int levels, double lo0, double lo1, double lo2, double hi0, double hi1,
                                 double hi2)
{
    const int64_t n_leaves = int64_t(1) << levels, n_nodes = 2 * n_leaves - 1;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    int level = 0;
    while ((int64_t(1) << (level + 1)) - 1 <= n) ++level;
    double blo[3] = {lo0, lo1, lo2}, bhi[3] = {hi0, hi1, hi2};
    const uint64_t path = (uint64_t)(n + 1);
    for (int l = 0; l < level; ++l) {  // walk down from the root
        const int ax = l % 3;
        const double mid = 0.5 * (blo[ax] + bhi[ax]);
        const int right = (int)((path >> (level - 1 - l)) & 1);
        if (right) blo[ax] = mid;
        else bhi[ax] = mid;
    }
    if (level < levels) {
        const int ax = level % 3;
        t.axis[n] = ax;
        t.split[n] = 0.5 * (blo[ax] + bhi[ax]);
        t.left[n] = (int32_t)(2 * n + 1);
        t.leaf[n] = -1;
    } else {
        const int64_t l = n - (n_leaves - 1);
        t.axis[n] = -1;
        t.split[n] = 0.0;
        t.left[n] = -1;
        t.leaf[n] = (int32_t)l;
        t.leaf_node[l] = (int32_t)n;
        for (int d = 0; d < 3; ++d) {
            t.lo[3 * l + d] = blo[d];
            t.hi[3 * l + d] = bhi[d];
        }
        t.init[l] = 0;
    }
    if (n == 0) {
        t.counts[0] = (int32_t)n_nodes;
        t.counts[1] = (int32_t)n_leaves;
    }
}

// ---------------------------------------------------------------------------------
// point location: left where p[axis] < split, else right; child indices exceed their
// parent's, so a walk ends within max_nodes steps. The oldest nodes, the top of the tree,
// are staged in LDS by every work group (one 8-byte entry per node, indices below
// kLocStaged: the whole tree while it has no more nodes than that), so a walk costs one
// LDS read per level there; below them a node's axis, split, left child and leaf index
// are loaded from global memory together (one memory round trip per level). Each thread
// walks kLocPer samples side by side, so their reads overlap, and issues the next tile's
// first loads before it walks the current one. After the first round a sample resumes
// from the node it reached in the previous round (node_of), which is still its leaf
// unless that leaf was split: its position is read only when it has to move, and its
// node index is written only when it changes.
//
// A staged entry holds the split rounded up to FP32: for an FP32 coordinate p and an FP64
// split s, p < s exactly when p < f, f the least FP32 value not below s (every FP32 value
// below s is at most the greatest one below f), so the walk takes the FP64 comparison's
// branch with an FP32 comparison.
// ---------------------------------------------------------------------------------
constexpr int kLocThreads = 512;
constexpr int kLocPer = 4;                       // samples per thread per tile
constexpr int kLocTile = kLocThreads * kLocPer;  // samples per work group per tile
constexpr int kLocStaged = 4096;                 // nodes staged in LDS (32 KB)
constexpr int kLocMaxGroups = 256 * 4;           // 4 work groups per CU
constexpr int32_t kUnstaged = INT32_MIN;         // an inner node whose child index does not fit the code

struct alignas(8) StagedNode {
    float split;   // the split rounded up to FP32
    int32_t code;  // inner node: 4 left + axis; leaf: -(leaf index) - 1; or kUnstaged
};

__device__ __forceinline__ float round_up_f32(double s)
{
    float f = (float)s;
    if ((double)f < s) f = __int_as_float(__float_as_int(f) + (f >= 0.0f ? 1 : -1));
    return f;
}

// the loads that start a tile: the positions when every sample starts at the root, else
// the nodes the samples reached before (a lane past the end loads the last sample's)
template <bool FromRoot>
__device__ __forceinline__ void loc_first_loads(const float* __restrict__ smp, const int32_t* __restrict__ node_of,
                                                int64_t N, int64_t b, float (&p0)[kLocPer], float (&p1)[kLocPer],
                                                float (&p2)[kLocPer], int32_t (&pn)[kLocPer])
{
#pragma unroll
    for (int r = 0; r < kLocPer; ++r) {
        const int64_t ic = min(b + r * kLocThreads, N - 1);
        if (FromRoot) {
            p0[r] = smp[3 * N + ic];
            p1[r] = smp[4 * N + ic];
            p2[r] = smp[5 * N + ic];
        } else {
            pn[r] = node_of[ic];
        }
    }
}

template <bool FromRoot>
__global__ __launch_bounds__(kLocThreads) void locate_kernel(TreePtrs t, const float* __restrict__ smp, int64_t N,
                                                             int32_t* __restrict__ node_of,
                                                             int32_t* __restrict__ leaf_of)
{
    __shared__ StagedNode top[kLocStaged];
    const int32_t ns = max(1, min(min(t.counts[0], t.max_nodes), kLocStaged));
    {
        constexpr int kPer = kLocStaged / kLocThreads;
        const int jn = (ns + kLocThreads - 1) / kLocThreads;  // the same in every lane
        int32_t ax[kPer], lf[kPer], lv[kPer];
        double sp[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {  // all loads first, then the LDS writes
            if (j >= jn) break;
            const int k = min(j * kLocThreads + (int)threadIdx.x, ns - 1);
            ax[j] = t.axis[k];
            lf[j] = t.left[k];
            lv[j] = t.leaf[k];
            sp[j] = t.split[k];
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            if (j >= jn) break;
            const int k = j * kLocThreads + (int)threadIdx.x;
            const int32_t code = ax[j] < 0 ? -lv[j] - 1 : (lf[j] < (1 << 29) ? 4 * lf[j] + ax[j] : kUnstaged);
            if (k < ns) top[k] = StagedNode{round_up_f32(sp[j]), code};
        }
    }
    __syncthreads();
    // a lane past the end walks the last sample's path again and stores nothing
    const int64_t stride = (int64_t)gridDim.x * kLocTile;
    int64_t base = (int64_t)blockIdx.x * kLocTile + threadIdx.x;
    float p0[kLocPer], p1[kLocPer], p2[kLocPer];  // first loads of the next tile
    int32_t pn[kLocPer];
    if (base < N) loc_first_loads<FromRoot>(smp, node_of, N, base, p0, p1, p2, pn);
    for (; base < N; base += stride) {
        int32_t n[kLocPer], n0[kLocPer];
        float q0[kLocPer], q1[kLocPer], q2[kLocPer];
        if (FromRoot) {
#pragma unroll
            for (int r = 0; r < kLocPer; ++r) {
                n0[r] = 0;
                q0[r] = p0[r];
                q1[r] = p1[r];
                q2[r] = p2[r];
            }
        } else {
#pragma unroll
            for (int r = 0; r < kLocPer; ++r) n0[r] = pn[r];
        }
        if (base + stride < N) loc_first_loads<FromRoot>(smp, node_of, N, base + stride, p0, p1, p2, pn);
        if (!FromRoot) {
            // a sample at an inner node moves: only then is its position read
            int32_t c[kLocPer];
#pragma unroll
            for (int r = 0; r < kLocPer; ++r) c[r] = top[min(n0[r], ns - 1)].code;
#pragma unroll
            for (int r = 0; r < kLocPer; ++r) {
                const bool staged = n0[r] < ns && c[r] != kUnstaged;
                const bool inner = staged ? c[r] >= 0 : t.axis[n0[r]] >= 0;
                const int64_t ic = min(base + r * kLocThreads, N - 1);
                q0[r] = q1[r] = q2[r] = 0.0f;
                if (inner) {
                    q0[r] = smp[3 * N + ic];
                    q1[r] = smp[4 * N + ic];
                    q2[r] = smp[5 * N + ic];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < kLocPer; ++r) n[r] = n0[r];
        // the staged levels: a step per LDS read
        for (int32_t s = 0; s <= ns; ++s) {
            bool more = false;
            StagedNode e[kLocPer];
#pragma unroll
            for (int r = 0; r < kLocPer; ++r) e[r] = top[min(n[r], ns - 1)];
#pragma unroll
            for (int r = 0; r < kLocPer; ++r) {
                const bool go = n[r] < ns && e[r].code >= 0;
                const float t01 = (e[r].code & 1) ? q1[r] : q0[r];
                const float pa = (e[r].code & 2) ? q2[r] : t01;
                const int32_t to = (e[r].code >> 2) + (pa < e[r].split ? 0 : 1);
                n[r] = go ? to : n[r];
                more |= go;
            }
            if (!more) break;
        }
        // the levels below: a step per global round trip (only where a walk left the
        // staged nodes, so that the other waves never wait for the next tile's loads)
        int32_t lv[kLocPer];
        bool staged[kLocPer], below = false;
#pragma unroll
        for (int r = 0; r < kLocPer; ++r) {
            const int32_t c = top[min(n[r], ns - 1)].code;
            staged[r] = n[r] < ns && c != kUnstaged;  // then a leaf
            lv[r] = -c - 1;
            below |= !staged[r];
        }
        if (below) {
            int32_t ax[kLocPer], lf[kLocPer];
            double sp[kLocPer];
#pragma unroll
            for (int r = 0; r < kLocPer; ++r) {
                ax[r] = -1;
                lf[r] = -1;
                sp[r] = 0.0;
                if (!staged[r]) {
                    ax[r] = t.axis[n[r]];
                    lf[r] = t.left[n[r]];
                    sp[r] = t.split[n[r]];
                    lv[r] = t.leaf[n[r]];
                }
            }
            for (int32_t s = 0; s < t.max_nodes; ++s) {
                // the loads above and below complete together at these empty statements
                // (the compiler would otherwise issue the later ones only after the axis
                // came back)
#pragma unroll
                for (int r = 0; r < kLocPer; ++r)
                    asm volatile("" ::"v"(ax[r]), "v"(lf[r]), "v"(sp[r]), "v"(lv[r]));
                bool more = false;
#pragma unroll
                for (int r = 0; r < kLocPer; ++r) {
                    if (ax[r] >= 0) {
                        const float pa = ax[r] == 0 ? q0[r] : (ax[r] == 1 ? q1[r] : q2[r]);
                        n[r] = (double)pa < sp[r] ? lf[r] : lf[r] + 1;
                        ax[r] = t.axis[n[r]];
                        lf[r] = t.left[n[r]];
                        sp[r] = t.split[n[r]];
                        lv[r] = t.leaf[n[r]];
                        more = true;
                    }
                }
                if (!more) break;
            }
        }
#pragma unroll
        for (int r = 0; r < kLocPer; ++r) {
            const int64_t i = base + r * kLocThreads;
            if (i >= N) continue;
            if (FromRoot || n[r] != n0[r]) node_of[i] = n[r];
            leaf_of[i] = lv[r];
        }
    }
}

// ---------------------------------------------------------------------------------
// stable LSD radix sort of (leaf index, sample index) by leaf index, 8 bits per pass
// ---------------------------------------------------------------------------------
// the valid lanes of the wave whose digit equals this lane's (meaningful for valid lanes):
// one comparison when every valid lane holds the same digit, as in runs of samples of one
// leaf, else one ballot per digit bit
__device__ __forceinline__ uint64_t digit_peers(int digit, bool valid)
{
    const uint64_t vm = __ballot(valid);
    const int d0 = __builtin_amdgcn_readfirstlane(digit);
    if (__all(!valid || digit == d0)) return vm;
    uint64_t peers = vm;
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        const uint64_t m = __ballot((digit >> b) & 1);
        peers &= ((digit >> b) & 1) ? m : ~m;
    }
    return peers;
}

__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const int32_t* __restrict__ keys, int64_t N,
                                                                  int shift, int32_t* __restrict__ hist, int B)
{
    __shared__ int32_t h[kRadix];
    h[threadIdx.x] = 0;
    __syncthreads();
    // lanes with equal digits (found by 8 ballots) add their count once: the keys of a
    // tile are mostly equal when the samples arrive grouped, and LDS atomics on one
    // address serialise
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    int32_t kv[kSortItems];  // the thread's keys, loaded together
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t i = base + (int64_t)it * kSortThreads + threadIdx.x;
        kv[it] = i < N ? keys[i] : 0;
    }
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t i = base + (int64_t)it * kSortThreads + threadIdx.x;
        const bool valid = i < N;
        const int digit = valid ? (kv[it] >> shift) & (kRadix - 1) : 0;
        const uint64_t peers = digit_peers(digit, valid);
        if (valid && (peers & lt) == 0) atomicAdd(&h[digit], __popcll(peers));
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * B + blockIdx.x] = h[threadIdx.x];
}

// Exclusive prefix sum of n int32 counts in three launches: tile sums (kScanTile
// entries per work group), an exclusive scan of the tile sums by one work group, and the
// scan of each tile from its base.
constexpr int kScanPer = 16;
constexpr int kScanTile = 256 * kScanPer;

__device__ __forceinline__ int32_t block_exclusive_scan_256(int32_t v, int32_t& total)
{
    __shared__ int32_t wsum[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int32_t before = 0;
    for (int q = 0; q < w; ++q) before += wsum[q];
    total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    return before + x - v;
}

__global__ __launch_bounds__(256) void scan_tile_sums_kernel(const int32_t* __restrict__ v, int64_t n,
                                                             int32_t* __restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int32_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q)
        if (base + q < n) s += v[base + q];
    int32_t total;
    (void)block_exclusive_scan_256(s, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void scan_sums_kernel(int32_t* __restrict__ v, int64_t n)
{
    __shared__ int64_t part[1024];
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t a = min(n, (int64_t)threadIdx.x * chunk), b = min(n, a + chunk);
    int64_t s = 0;
    for (int64_t i = a; i < b; ++i) s += v[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // inclusive scan of the partial sums
        const int64_t add = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t run = part[threadIdx.x] - s;
    for (int64_t i = a; i < b; ++i) {
        const int64_t c = v[i];
        v[i] = (int32_t)run;
        run += c;
    }
}

__global__ __launch_bounds__(256) void scan_apply_kernel(int32_t* __restrict__ v, int64_t n,
                                                         const int32_t* __restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int32_t x[kScanPer];
    int32_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        x[q] = base + q < n ? v[base + q] : 0;
        s += x[q];
    }
    int32_t total;
    int32_t run = sums[blockIdx.x] + block_exclusive_scan_256(s, total);
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        if (base + q < n) v[base + q] = run;
        run += x[q];
    }
}

// Each block scatters its tile in index order: per 256-key step, a key's rank among the
// equal digits of its wave comes from 8 ballots (the tile's keys and values are loaded up
// front), the waves of the block are ordered by
// per-wave digit counts in LDS, and a running base per digit carries over the steps.
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(const int32_t* __restrict__ kin,
                                                                     const int32_t* __restrict__ vin, int64_t N,
                                                                     int shift, const int32_t* __restrict__ hist,
                                                                     int B, int32_t* __restrict__ kout,
                                                                     int32_t* __restrict__ vout)
{
    constexpr int W = kSortThreads / 64;
    __shared__ int32_t base[kRadix];
    __shared__ int32_t wcount[W][kRadix];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    base[tid] = hist[(int64_t)tid * B + blockIdx.x];
    for (int q = 0; q < W; ++q) wcount[q][tid] = 0;
    __syncthreads();
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int64_t tile = (int64_t)blockIdx.x * kSortTile;
    // the thread's keys and values, loaded together before the barriers of the steps
    int32_t kv[kSortItems], vv[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t i = tile + (int64_t)it * kSortThreads + tid;
        const bool valid = i < N;
        kv[it] = valid ? kin[i] : 0;
        vv[it] = valid ? (vin ? vin[i] : (int32_t)i) : 0;
    }
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t i = tile + (int64_t)it * kSortThreads + tid;
        const bool valid = i < N;
        const int32_t key = kv[it];
        const int32_t val = vv[it];
        const int digit = (key >> shift) & (kRadix - 1);
        const uint64_t peers = digit_peers(digit, valid);
        const int rank = __popcll(peers & lt);
        if (valid && rank == 0) wcount[w][digit] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int32_t before = base[digit];
            for (int q = 0; q < w; ++q) before += wcount[q][digit];
            const int64_t dst = (int64_t)before + rank;
            kout[dst] = key;
            vout[dst] = val;
        }
        __syncthreads();
        int32_t tot = 0;
        for (int q = 0; q < W; ++q) {
            tot += wcount[q][tid];
            wcount[q][tid] = 0;
        }
        base[tid] += tot;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------
// the order by leaf after a round's splits follows from the previous round's: a sample
// stays in its leaf, or goes to the left child, which keeps the parent's leaf index, or to
// the right child, whose index is at least the previous leaf count and grows with the
// parent's. So the samples now below that count keep their relative order, and the others
// follow them in theirs: a stable partition of the previous permutation (two launches and
// a one-group scan of the tiles' counts) takes the place of the radix sort.
// ---------------------------------------------------------------------------------

// cnt[b] = the samples of tile b (in the previous order) now in a leaf >= L_old; cnt[B] = 0
__global__ __launch_bounds__(kSortThreads) void part_count_kernel(const int32_t* __restrict__ perm,
                                                                  const int32_t* __restrict__ leaf_of, int64_t N,
                                                                  int32_t L_old, int32_t* __restrict__ cnt, int B)
{
    const int64_t tile = (int64_t)blockIdx.x * kSortTile;
    int32_t pv[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t i = tile + (int64_t)it * kSortThreads + threadIdx.x;
        pv[it] = perm[min(i, N - 1)];
    }
    int32_t c = 0;
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t i = tile + (int64_t)it * kSortThreads + threadIdx.x;
        c += (i < N && leaf_of[pv[it]] >= L_old) ? 1 : 0;
    }
    int32_t total;
    (void)block_exclusive_scan_256(c, total);
    if (threadIdx.x == 0) {
        cnt[blockIdx.x] = total;
        if (blockIdx.x == 0) cnt[B] = 0;
    }
}

// after the exclusive scan of cnt (cnt[B] = all such samples): position j of the previous
// order goes to j - t_j, or to N - cnt[B] + t_j if its new leaf is >= L_old, t_j being the
// number of such samples before j
__global__ __launch_bounds__(kSortThreads) void part_scatter_kernel(const int32_t* __restrict__ perm,
                                                                    const int32_t* __restrict__ leaf_of, int64_t N,
                                                                    int32_t L_old, const int32_t* __restrict__ cnt,
                                                                    int B, int32_t* __restrict__ kout,
                                                                    int32_t* __restrict__ vout)
{
    constexpr int W = kSortThreads / 64;
    __shared__ int32_t wt[W];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int64_t tile = (int64_t)blockIdx.x * kSortTile;
    const int64_t first_up = N - (int64_t)cnt[B];
    int32_t pv[kSortItems], kv[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t i = tile + (int64_t)it * kSortThreads + threadIdx.x;
        pv[it] = perm[min(i, N - 1)];
    }
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) kv[it] = leaf_of[pv[it]];
    int64_t run = cnt[blockIdx.x];  // such samples before the current step
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t i = tile + (int64_t)it * kSortThreads + threadIdx.x;
        const bool valid = i < N, up = valid && kv[it] >= L_old;
        const uint64_t m = __ballot(up);
        if (lane == 0) wt[w] = __popcll(m);
        __syncthreads();
        int64_t tj = run + __popcll(m & lt);
        int32_t all = 0;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            tj += q < w ? wt[q] : 0;
            all += wt[q];
        }
        if (valid) {
            const int64_t dst = up ? first_up + tj : i - tj;
            kout[dst] = kv[it];
            vout[dst] = pv[it];
        }
        run += all;
        __syncthreads();
    }
}

// off[l] = first sorted position of leaf l (off[L] = N), for leaves 0..L
__global__ void segment_kernel(const int32_t* __restrict__ keys, int64_t N, int32_t L, int64_t* __restrict__ off)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (N == 0) {
        if (i <= L) off[i] = 0;
        return;
    }
    if (i >= N) return;
    const int32_t k = keys[i], kp = i > 0 ? keys[i - 1] : -1;
    for (int32_t l = kp + 1; l <= k; ++l) off[l] = i;
    if (i == N - 1)
        for (int32_t l = k + 1; l <= L; ++l) off[l] = N;
}

// ---------------------------------------------------------------------------------
// split statistics: one work group of kStatThreads per leaf of the round with more than c
// samples (16 waves, so that the few large leaves of the first rounds keep enough loads in
// flight); FP64 sums reduced in a fixed order (lanes by butterfly, then the waves in order)
// ---------------------------------------------------------------------------------
constexpr int kStatThreads = 1024;

__global__ __launch_bounds__(kStatThreads) void split_stats_kernel(const float* __restrict__ smp, int64_t N,
                                                          const int32_t* __restrict__ perm,
                                                          const int64_t* __restrict__ off, int32_t L, int32_t c,
                                                          const int32_t* __restrict__ act, int32_t* __restrict__ want,
                                                          int32_t* __restrict__ sax, double* __restrict__ spos)
{
    constexpr int W = kStatThreads / 64;
    __shared__ double ls1[W][3], lsq[W][3];
    __shared__ float lmn[W][3], lmx[W][3];
    const int l = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (l >= L) return;
    const int64_t a = off[l], b = off[l + 1], M = b - a;
    if (!act[l] || M <= c) {
        if (threadIdx.x == 0) want[l] = 0;
        return;
    }
    double s1[3] = {0, 0, 0}, sq[3] = {0, 0, 0};
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    // the positions are gathered through the sort's permutation: four of a thread's
    // samples are loaded together (indices clamped into the leaf, so every load is in
    // bounds) and then added in the thread's sample order
    constexpr int U = 4;
    int32_t idx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) idx[u] = perm[min(a + threadIdx.x + u * kStatThreads, b - 1)];
    for (int64_t j0 = a + threadIdx.x; j0 < b; j0 += U * kStatThreads) {
        float xs[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int d = 0; d < 3; ++d) xs[u][d] = smp[(3 + d) * N + idx[u]];
        // the next step's indices are on their way while these positions are added
        const int64_t jn = j0 + U * kStatThreads;
        if (jn < b) {
#pragma unroll
            for (int u = 0; u < U; ++u) idx[u] = perm[min(jn + u * kStatThreads, b - 1)];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (j0 + u * kStatThreads >= b) break;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const float xf = xs[u][d];
                const double x = (double)xf;
                s1[d] += x;
                sq[d] += x * x;
                mn[d] = fminf(mn[d], xf);
                mx[d] = fmaxf(mx[d], xf);
            }
        }
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            s1[d] += __shfl_xor(s1[d], o);
            sq[d] += __shfl_xor(sq[d], o);
            mn[d] = fminf(mn[d], __shfl_xor(mn[d], o));
            mx[d] = fmaxf(mx[d], __shfl_xor(mx[d], o));
        }
    }
    if (lane == 0)
        for (int d = 0; d < 3; ++d) {
            ls1[w][d] = s1[d];
            lsq[w][d] = sq[d];
            lmn[w][d] = mn[d];
            lmx[w][d] = mx[d];
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int d = 0; d < 3; ++d) {  // the waves' results in wave order
            s1[d] = ls1[0][d];
            sq[d] = lsq[0][d];
            mn[d] = lmn[0][d];
            mx[d] = lmx[0][d];
            for (int q = 1; q < W; ++q) {
                s1[d] += ls1[q][d];
                sq[d] += lsq[q][d];
                mn[d] = fminf(mn[d], lmn[q][d]);
                mx[d] = fmaxf(mx[d], lmx[q][d]);
            }
        }
        const double Md = (double)M;
        int ax = 0;
        double best = -1.0;
        for (int d = 0; d < 3; ++d) {
            const double mean = s1[d] / Md;
            const double var = sq[d] / Md - mean * mean;
            if (var > best) {
                best = var;
                ax = d;
            }
        }
        const double split = s1[ax] / Md;
        want[l] = ((double)mn[ax] < split && split <= (double)mx[ax]) ? 1 : 0;
        sax[l] = ax;
        spos[l] = split;
    }
}

// ---------------------------------------------------------------------------------
// split decisions in leaf order by one work group; ctl[0] = splits made, ctl[1] |= 1
// when the capacity stopped some
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void split_decide_kernel(TreePtrs t, int32_t L, const int32_t* __restrict__ want,
                                                            const int32_t* __restrict__ sax,
                                                            const double* __restrict__ spos,
                                                            int32_t* __restrict__ act,
                                                            int32_t* __restrict__ parent_of, int32_t* __restrict__ ctl)
{
    __shared__ int32_t part[1024];
    const int32_t nodes = t.counts[0], leaves = t.counts[1];
    const int32_t chunk = (L + 1023) / 1024;
    const int32_t a = min(L, (int32_t)threadIdx.x * chunk), b = min(L, a + chunk);
    int32_t s = 0;
    for (int32_t l = a; l < b; ++l) s += want[l];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int32_t add = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    const int32_t total = part[1023];
    const int32_t cap = min((t.max_nodes - nodes) / 2, t.max_leaves - leaves);
    const int32_t n_split = min(total, max(cap, 0));
    int32_t rank = part[threadIdx.x] - s;
    for (int32_t l = a; l < b; ++l) {
        const bool go = want[l] && rank < n_split;
        if (want[l]) ++rank;
        if (!go) {
            act[l] = 0;
            continue;
        }
        const int32_t rk = rank - 1;
        const int32_t r = leaves + rk, Ln = nodes + 2 * rk;
        const int32_t n = t.leaf_node[l];
        const int ax = sax[l];
        const double sp = spos[l];
        t.axis[n] = ax;
        t.split[n] = sp;
        t.left[n] = Ln;
        t.leaf[n] = -1;
        for (int q = 0; q < 2; ++q) {
            t.axis[Ln + q] = -1;
            t.left[Ln + q] = -1;
            t.split[Ln + q] = 0.0;
        }
        t.leaf[Ln] = l;
        t.leaf[Ln + 1] = r;
        t.leaf_node[l] = Ln;
        t.leaf_node[r] = Ln + 1;
        for (int d = 0; d < 3; ++d) {
            t.lo[3 * r + d] = t.lo[3 * l + d];
            t.hi[3 * r + d] = t.hi[3 * l + d];
        }
        t.hi[3 * l + ax] = sp;
        t.lo[3 * r + ax] = sp;
        t.init[r] = t.init[l];
        parent_of[rk] = l;
        act[l] = 1;
        act[r] = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        t.counts[0] = nodes + 2 * n_split;
        t.counts[1] = leaves + n_split;
        ctl[0] = n_split;
        ctl[1] |= total > n_split ? 1 : 0;
    }
}

// the new leaf r = leaves_before + rank copies its parent's mixture and state
__global__ void copy_leaves_kernel(int32_t leaves_before, int32_t n_split, const int32_t* __restrict__ parent_of,
                                   int K, MixPtrs mix, StatePtrs st)
{
    const int rk = blockIdx.x;
    if (rk >= n_split) return;
    const int64_t r = leaves_before + rk, l = parent_of[rk];
    for (int q = threadIdx.x; q < 38 * K + 2; q += blockDim.x) {
        if (q < K) mix.pi[r * K + q] = mix.pi[l * K + q];
        else if (q < 4 * K) mix.mud[r * 3 * K + q - K] = mix.mud[l * 3 * K + q - K];
        else if (q < 7 * K) mix.mux[r * 3 * K + q - 4 * K] = mix.mux[l * 3 * K + q - 4 * K];
        else if (q < 22 * K) mix.cov[r * 15 * K + q - 7 * K] = mix.cov[l * 15 * K + q - 7 * K];
        else if (q < 23 * K) st.s0[r * K + q - 22 * K] = st.s0[l * K + q - 22 * K];
        else if (q < 38 * K) st.s2[r * 15 * K + q - 23 * K] = st.s2[l * 15 * K + q - 23 * K];
        else if (q == 38 * K) st.sw[r] = st.sw[l];
        else st.step[r] = st.step[l];
    }
}

__global__ void set_active_kernel(int32_t* __restrict__ act, const int32_t* __restrict__ counts, int32_t max_leaves,
                                  int32_t* __restrict__ ctl)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < min(counts[1], max_leaves)) act[l] = 1;
    if (l == 0) ctl[0] = ctl[1] = 0;
}

// Work groups go to the eight XCDs in turn (group b to XCD b % 8), each XCD with its own
// L2. The groups of one XCD take consecutive ranges of the output, so that a source line
// a run of gathered samples only partly covers is fetched into one L2, not into two.
__device__ __forceinline__ int64_t xcd_block_order(int64_t b, int64_t nb)
{
    const int64_t x = b % 8, q = b / 8, per = nb / 8, extra = nb % 8;
    return x * per + (x < extra ? x : extra) + q;
}

__global__ void gather_kernel(const float* __restrict__ smp, int64_t N, const int32_t* __restrict__ perm,
                              float* __restrict__ out)
{
    const int64_t j = xcd_block_order(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int32_t i = perm[j];
#pragma unroll
    for (int a = 0; a < 7; ++a) out[a * N + j] = smp[a * N + i];
}

// Initial mixture of an uninitialised leaf with at least min_init samples, one thread
// per component: n_dir = min(8, K) directions at the cube vertices (signs of x, y, z,
// positive first), n_pos = ceil(K / n_dir) positions along the longest sides (two:
// centre -+ d/4; four: a 2x2 pattern; more: evenly), directional variance 2 pi / 8,
// positional variance r^2 / chi2_3^-1(0.9) with r = 2 d / n_pos, weights 1/K; the
// Robbins-Monro state starts at zero.
__global__ void init_leaves_kernel(TreePtrs t, int32_t L, const int64_t* __restrict__ off, int32_t min_init, int K,
                                   MixPtrs mix, StatePtrs st)
{
    const int l = blockIdx.x;
    if (l >= L || t.init[l] || off[l + 1] - off[l] < min_init) return;
    const double chi2_3_inv_090 = 6.251388631170325;
    const int n_dir = K < 8 ? K : 8;
    const int n_pos = (K + n_dir - 1) / n_dir;
    double size[3], centre[3], d = 0.0;
    for (int a = 0; a < 3; ++a) {
        size[a] = t.hi[3 * l + a] - t.lo[3 * l + a];
        centre[a] = t.lo[3 * l + a] + 0.5 * size[a];
        d = fmax(d, size[a]);
    }
    int order[3] = {0, 1, 2};
    for (int i = 1; i < 3; ++i)
        for (int j = i; j > 0 && size[order[j]] > size[order[j - 1]]; --j) {
            const int tmp = order[j];
            order[j] = order[j - 1];
            order[j - 1] = tmp;
        }
    const double r = 2.0 * d / n_pos;
    const double inv_sqrt3 = 1.0 / sqrt(3.0);
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const int s = k / n_dir, v = k % n_dir;
        double o[3] = {0.0, 0.0, 0.0};
        if (n_pos == 2) {
            o[order[0]] = (s == 0 ? -1.0 : 1.0) * d / 4.0;
        } else if (n_pos == 4) {
            o[order[0]] = (s % 2 == 0 ? -1.0 : 1.0) * d / 4.0;
            o[order[1]] = (s / 2 == 0 ? -1.0 : 1.0) * d / 4.0;
        } else if (n_pos > 1) {
            o[order[0]] = ((s + 0.5) / n_pos - 0.5) * d;
        }
        const int64_t g = (int64_t)l * K + k;
        for (int a = 0; a < 3; ++a) mix.mux[3 * g + a] = centre[a] + o[a];
        mix.mud[3 * g + 0] = ((v >> 2) & 1 ? -1.0 : 1.0) * inv_sqrt3;
        mix.mud[3 * g + 1] = ((v >> 1) & 1 ? -1.0 : 1.0) * inv_sqrt3;
        mix.mud[3 * g + 2] = (v & 1 ? -1.0 : 1.0) * inv_sqrt3;
        for (int q = 0; q < 15; ++q) mix.cov[15 * g + q] = 0.0;
        mix.cov[15 * g + tri(0, 0)] = mix.cov[15 * g + tri(1, 1)] = 2.0 * kPi / 8.0;
        for (int a = 0; a < 3; ++a) mix.cov[15 * g + tri(2 + a, 2 + a)] = r * r / chi2_3_inv_090;
        mix.pi[g] = 1.0 / K;
        st.s0[g] = 0.0;
        for (int q = 0; q < 15; ++q) st.s2[15 * g + q] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st.sw[l] = 0.0;
        st.step[l] = 0;
        t.init[l] = 1;
    }
}

// workspace of a refinement
struct TreeLayout {
    size_t nodeof, keys0, keys1, vals0, vals1, hist, tsum, off, act, want, sax, spos, parent, ctl, total;
    int B;
};

inline TreeLayout tree_layout(int64_t N, int32_t max_leaves)
{
    TreeLayout L{};
    const int64_t n = N > 0 ? N : 1;
    L.B = (int)((n + kSortTile - 1) / kSortTile);
    size_t p = 0;
    auto take = [&](size_t bytes) {
        const size_t at = p;
        p = align256(p + bytes);
        return at;
    };
    L.nodeof = take(n * 4);
    L.keys0 = take(n * 4);
    L.keys1 = take(n * 4);
    L.vals0 = take(n * 4);
    L.vals1 = take(n * 4);
    L.hist = take((size_t)kRadix * L.B * 4);
    L.tsum = take(((size_t)kRadix * L.B + kScanTile - 1) / kScanTile * 4);
    L.off = take(((size_t)max_leaves + 1) * 8);
    L.act = take((size_t)max_leaves * 4);
    L.want = take((size_t)max_leaves * 4);
    L.sax = take((size_t)max_leaves * 4);
    L.spos = take((size_t)max_leaves * 8);
    L.parent = take((size_t)max_leaves * 4);
    L.ctl = take(4 * 4);
    L.total = p;
    return L;
}

static TreePtrs tree_ptrs(const sdmm_tree* t)
{
    return TreePtrs{t->max_nodes, t->max_leaves, t->counts, t->axis, t->left, t->leaf, t->split,
                    t->leaf_node, t->lo, t->hi, t->init};
}

static bool tree_ok(const sdmm_tree* t)
{
    return t && t->max_leaves >= 1 && t->max_nodes >= 2 * t->max_leaves - 1 && t->counts && t->axis && t->left &&
           t->leaf && t->split && t->leaf_node && t->lo && t->hi && t->init;
}

static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }

}  // namespace sdmm

using namespace sdmm;

extern "C" int sdmm_tree_init(const sdmm_tree* tree, int32_t depth, const double* lo, const double* hi, void* stream)
{
    if (!tree_ok(tree) || !lo || !hi || depth < 0 || depth > 6) return SDMM_EINVAL;
    const int levels = 3 * depth;
    const int64_t n_leaves = int64_t(1) << levels, n_nodes = 2 * n_leaves - 1;
    if (n_leaves > tree->max_leaves || n_nodes > tree->max_nodes) return SDMM_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (!(lo[d] < hi[d])) return SDMM_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    tree_init_kernel<<<blocks_for(n_nodes, 256), 256, 0, s>>>(tree_ptrs(tree), levels, lo[0], lo[1], lo[2], hi[0],
                                                             hi[1], hi[2]);
    return check(hipGetLastError());
}

extern "C" size_t sdmm_tree_workspace_size(int64_t n_samples, int32_t max_leaves)
{
    if (n_samples < 0 || max_leaves < 1) return 0;
    return tree_layout(n_samples, max_leaves).total;
}

extern "C" int sdmm_tree_refine(const sdmm_tree* tree, const float* samples, int64_t n_samples,
                                int32_t split_threshold, int32_t min_init, const sdmm_mixtures* mix,
                                const sdmm_em_state* state, float* sorted_out, int64_t* cell_offsets_out,
                                int32_t* n_leaves_out, int32_t* status_out, void* workspace,
                                size_t workspace_bytes, void* stream)
{
    if (!tree_ok(tree) || n_samples < 0 || (n_samples > 0 && (!samples || !sorted_out)) || split_threshold < 1 ||
        min_init < 0 || !mix || !state || !cell_offsets_out || !n_leaves_out || !workspace)
        return SDMM_EINVAL;
    if (n_samples > INT32_MAX) return SDMM_EINVAL;  // sample indices are int32
    if (mix->n_cells != tree->max_leaves || mix->K < 1 || mix->K > kMaxK || !mix->weights || !mix->mean_dir ||
        !mix->mean_pos || !mix->cov || !state->s0 || !state->s2 || !state->sw || !state->step)
        return SDMM_EINVAL;
    const int64_t N = n_samples;
    const TreeLayout TL = tree_layout(N, tree->max_leaves);
    if (workspace_bytes < TL.total) return SDMM_ENOWORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char* ws = reinterpret_cast<char*>(workspace);
    int32_t* nodeof = reinterpret_cast<int32_t*>(ws + TL.nodeof);
    int32_t* k0 = reinterpret_cast<int32_t*>(ws + TL.keys0);
    int32_t* k1 = reinterpret_cast<int32_t*>(ws + TL.keys1);
    int32_t* v0 = reinterpret_cast<int32_t*>(ws + TL.vals0);
    int32_t* v1 = reinterpret_cast<int32_t*>(ws + TL.vals1);
    int32_t* hist = reinterpret_cast<int32_t*>(ws + TL.hist);
    int32_t* tsum = reinterpret_cast<int32_t*>(ws + TL.tsum);
    int64_t* off = reinterpret_cast<int64_t*>(ws + TL.off);
    int32_t* act = reinterpret_cast<int32_t*>(ws + TL.act);
    int32_t* want = reinterpret_cast<int32_t*>(ws + TL.want);
    int32_t* sax = reinterpret_cast<int32_t*>(ws + TL.sax);
    double* spos = reinterpret_cast<double*>(ws + TL.spos);
    int32_t* parent = reinterpret_cast<int32_t*>(ws + TL.parent);
    int32_t* ctl = reinterpret_cast<int32_t*>(ws + TL.ctl);
    const TreePtrs tp = tree_ptrs(tree);
    const MixPtrs mp{mix->weights, mix->mean_dir, mix->mean_pos, mix->cov};
    const StatePtrs sp{state->s0, state->s2, state->sw, state->step};
    const int K = mix->K;
    int rc;

    // the words read back once per round land in pinned memory (a pageable destination
    // would be staged by the runtime), one buffer per host thread, kept for its lifetime
    thread_local int32_t* pinned = nullptr;
    if (!pinned && (rc = check(hipHostMalloc((void**)&pinned, 4 * sizeof(int32_t), hipHostMallocPortable)))) {
        pinned = nullptr;
        return rc;
    }
    int32_t* counts = pinned;
    int32_t* c2 = pinned + 2;

    // what needs no leaf count on the host is queued ahead of its readback, so that the GPU
    // works while the host waits: the location of every sample from the root, the active
    // flags (from the count on the device) and the first pass of the radix sort. Only the
    // workspace is written before the tree's counts are checked.
    const unsigned loc_groups = std::min<unsigned>(blocks_for(N, kLocTile), kLocMaxGroups);
    {  // the full location of every sample from the root is timed
        ScopedTimer tm(SDMM_TIMER_TREE, s);
        locate_kernel<true><<<loc_groups, kLocThreads, 0, s>>>(tp, samples, N, nodeof, k0);
    }
    set_active_kernel<<<blocks_for(tree->max_leaves, 256), 256, 0, s>>>(act, tree->counts, tree->max_leaves, ctl);
    // the first round's stable LSD radix sort from the sample order, 8 bits per pass
    const int32_t *kin = k0, *vin = nullptr;
    int32_t *kout = k1, *vout = v1;
    auto sort_pass = [&](int p) {
        radix_hist_kernel<<<TL.B, kSortThreads, 0, s>>>(kin, N, p * kRadixBits, hist, TL.B);
        const int64_t nh = (int64_t)kRadix * TL.B;
        const unsigned nt = (unsigned)((nh + kScanTile - 1) / kScanTile);
        scan_tile_sums_kernel<<<nt, 256, 0, s>>>(hist, nh, tsum);
        scan_sums_kernel<<<1, 1024, 0, s>>>(tsum, nt);
        scan_apply_kernel<<<nt, 256, 0, s>>>(hist, nh, tsum);
        radix_scatter_kernel<<<TL.B, kSortThreads, 0, s>>>(kin, vin, N, p * kRadixBits, hist, TL.B, kout, vout);
        kin = kout;
        vin = vout;
        kout = (kout == k1) ? k0 : k1;
        vout = (vout == v1) ? v0 : v1;
    };
    if (N > 0) sort_pass(0);
    if ((rc = check(hipMemcpyAsync(counts, tree->counts, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s))))
        return rc;
    if ((rc = check(hipStreamSynchronize(s)))) return rc;
    int32_t L = counts[1];
    if (L < 1 || L > tree->max_leaves || counts[0] < 1 || counts[0] > tree->max_nodes) return SDMM_EINVAL;
    {
        int bits = 1;
        while ((int64_t(1) << bits) < L) ++bits;
        const int passes = (bits + kRadixBits - 1) / kRadixBits;
        for (int p = 1; p < passes && N > 0; ++p) sort_pass(p);
    }

    const int32_t* sorted_vals = v0;
    int32_t L_old = L;  // the leaf count before the last round's splits
    for (int round = 0;; ++round) {
        if (round > 0 && N > 0) {
            // locate from the nodes reached before, then a stable partition of the
            // previous order (k0 holds the new leaves)
            locate_kernel<false><<<loc_groups, kLocThreads, 0, s>>>(tp, samples, N, nodeof, k0);
            int32_t* pout = (vin == v0) ? v1 : v0;
            part_count_kernel<<<TL.B, kSortThreads, 0, s>>>(vin, k0, N, L_old, hist, TL.B);
            scan_sums_kernel<<<1, 1024, 0, s>>>(hist, (int64_t)TL.B + 1);
            part_scatter_kernel<<<TL.B, kSortThreads, 0, s>>>(vin, k0, N, L_old, hist, TL.B, k1, pout);
            kin = k1;
            vin = pout;
        }
        sorted_vals = N > 0 ? vin : v0;
        segment_kernel<<<blocks_for(std::max<int64_t>(N, (int64_t)L + 1), 256), 256, 0, s>>>(kin, N, L, off);
        if (round == kMaxRounds) break;
        // statistics and decisions
        split_stats_kernel<<<L, kStatThreads, 0, s>>>(samples, N, vin, off, L, split_threshold, act, want, sax, spos);
        split_decide_kernel<<<1, 1024, 0, s>>>(tp, L, want, sax, spos, act, parent, ctl);
        if ((rc = check(hipMemcpyAsync(c2, ctl, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s)))) return rc;
        if ((rc = check(hipStreamSynchronize(s)))) return rc;
        if (c2[0] == 0) break;
        copy_leaves_kernel<<<c2[0], 64, 0, s>>>(L, c2[0], parent, K, mp, sp);
        L_old = L;
        L += c2[0];
    }
    if (N > 0) gather_kernel<<<blocks_for(N, 256), 256, 0, s>>>(samples, N, sorted_vals, sorted_out);
    if ((rc = check(hipMemcpyAsync(cell_offsets_out, off, ((size_t)L + 1) * 8, hipMemcpyDeviceToDevice, s))))
        return rc;
    init_leaves_kernel<<<L, 64, 0, s>>>(tp, L, off, min_init, K, mp, sp);
    if ((rc = check(hipMemcpyAsync(c2, ctl, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s)))) return rc;
    if ((rc = check(hipStreamSynchronize(s)))) return rc;
    *n_leaves_out = L;
    if (status_out) *status_out = c2[1];
    return check(hipGetLastError());
}
