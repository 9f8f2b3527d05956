// sbp_device.h -- device helpers shared by the gfx950 kernels: Philox4x32-10,
// index draws, f(x) = x ln x, wave64 reductions and the per-graph descriptor.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SBP_WAVE 64

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of the
// two-multiplier S-box with a Weyl key schedule.
// ---------------------------------------------------------------------------
struct Words4 {
    uint64_t w[4];
};

__device__ __forceinline__ void philox_block(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                             uint32_t k1, uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// Words W0..W3 from the blocks (a, b, base, tag) and (a, b, base + 1, tag).
__device__ __forceinline__ Words4 draw_words(uint64_t seed, uint32_t a, uint32_t b, uint32_t base, uint32_t tag) {
    Words4 W;
    uint32_t o[4];
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    philox_block(a, b, base, tag, k0, k1, o);
    W.w[0] = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
    W.w[1] = (uint64_t)o[2] | ((uint64_t)o[3] << 32);
    philox_block(a, b, base + 1u, tag, k0, k1, o);
    W.w[2] = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
    W.w[3] = (uint64_t)o[2] | ((uint64_t)o[3] << 32);
    return W;
}

// floor(W * n / 2^64): the high 64 bits of the 128-bit product.
__device__ __forceinline__ int64_t draw_idx(uint64_t W, uint64_t n) { return (int64_t)__umul64hi(W, n); }

// u = ((W >> 11) + 0.5) 2^-53 in (0, 1)
__device__ __forceinline__ double draw_unit(uint64_t W) {
    return ((double)(W >> 11) + 0.5) * 1.1102230246251565404236316680908203125e-16;
}

// f(x) = x ln x, f(0) = 0
__device__ __forceinline__ double xlogx(double x) { return x > 0.0 ? x * log(x) : 0.0; }

// Order-preserving rank of a merge score: floor(x 2^20), +inf last.
__device__ __forceinline__ int64_t merge_rank(double x) {
    if (!(x < 1e300)) return INT64_MAX;
    return (int64_t)floor(x * 1048576.0);
}

// ---------------------------------------------------------------------------
// wave64 helpers (fixed butterfly order, so sums are reproducible)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, SBP_WAVE);
    return x;
}
__device__ __forceinline__ int64_t wave_sum_i64(int64_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, SBP_WAVE);
    return x;
}
__device__ __forceinline__ int wave_sum_i32(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, SBP_WAVE);
    return x;
}
__device__ __forceinline__ int wave_max_i32(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, SBP_WAVE));
    return x;
}
__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}
// A DPP move of a double: both halves with the same control.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
// Sum over an aligned group of 8 lanes (half a DPP row): pairs, quads, then
// the mirrored half.  Each step adds the same two values on every lane, so the
// whole group ends with one identical sum.
__device__ __forceinline__ double grp8_sum(double x) {
    x += dpp_f64<0xB1>(x);   // quad_perm [1, 0, 3, 2]
    x += dpp_f64<0x4E>(x);   // quad_perm [2, 3, 0, 1]
    x += dpp_f64<0x141>(x);  // row_half_mirror
    return x;
}

// Sum over an aligned group of GS = 4, 8, 16 or 32 lanes: pairs, quads, the
// mirrored half row (8 and more), the mirrored row (16, 32), then the
// neighbouring row (32).  Each step adds the same two values on every lane (in
// either order), so the whole group ends with one identical sum.
template <int GS>
__device__ __forceinline__ double grp_sum(double x) {
    x += dpp_f64<0xB1>(x);   // quad_perm [1, 0, 3, 2]
    x += dpp_f64<0x4E>(x);   // quad_perm [2, 3, 0, 1]
    if (GS >= 8) x += dpp_f64<0x141>(x);  // row_half_mirror
    if (GS >= 16) x += dpp_f64<0x140>(x);  // row_mirror
    if (GS >= 32) x += __shfl_xor(x, 16, 64);
    return x;
}
template <int GS>
__device__ __forceinline__ int grp_sum_i32(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xf, 0xf, false);
    if (GS >= 8) x += __builtin_amdgcn_update_dpp(0, x, 0x141, 0xf, 0xf, false);
    if (GS >= 16) x += __builtin_amdgcn_update_dpp(0, x, 0x140, 0xf, 0xf, false);
    if (GS >= 32) x += __shfl_xor(x, 16, 64);
    return x;
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// Graph descriptor of a batched launch.  Every graph keeps its own arrays;
// union offsets place its vertices, blocks and edges in the shared buffers.
// ---------------------------------------------------------------------------
struct GDev {
    const int *out_ptr, *out_idx, *in_ptr, *in_idx;
    int *lab;             // working assignment [n]
    const int *leaf;      // vertices with at most SBP_LEAF_MAX edge ends
    const int *hub;       // the others
    int n, e, C, action;  // action of this step (ACT_*)
    int voff, boff;       // union vertex / block offsets
    long long eoff;       // union edge offset
    int n_leaf, n_hub;
    int merges;           // merges wanted in this merge phase
    int slot;             // engine slot of the graph
    unsigned long long seed;
    unsigned sweep, phase;
    double beta;
    int eps, n_batches, batch, proposals;
    // nullable: the sweep index is read from here instead of `sweep` (a
    // replayed graph), and the last batch's final step adds one to it
    unsigned *sweep_dev;
    // nullable: vertices with skip[v] > 0 (the hubs a hybrid sweep already
    // moved one at a time) take no part in this batch
    const int *skip;
    // nullable: M of this graph as a C x C table (graph-local ids), filled
    // for the step, so the sweep reads an entry with one load
    int *mdense;
};
__device__ __forceinline__ unsigned sweep_of(const GDev &g) { return g.sweep_dev ? *g.sweep_dev : g.sweep; }
// Whether vertex v belongs to this step's batch.
__device__ __forceinline__ bool in_batch(const GDev &g, int v) {
    return (v % g.n_batches) == g.batch && !(g.skip && g.skip[v] > 0);
}

// Per-step flat work lists: starts[g] is graph g's first item (graphs with
// no items in a list get an empty range at the right place).
struct StepMeta {
    const int *voff;     // union vertex starts (all graphs)
    const int *chstart;  // DL chunk starts
    const int *leaf;     // sweep items, vertices with <= SBP_LEAF_MAX ends
    const int *hub;      // sweep items, hubs
    const int *mblk;     // merge items (blocks of merging graphs)
    const int *mvtx;     // vertices of merging graphs
    const int *cblk;     // compaction items (blocks)
    const int *cvtx;     // vertices of compacting graphs
    int n_chunks, n_leaf, n_hub, n_mblk, n_mvtx, n_cblk, n_cvtx;
    int Ctot, maxC_merge, G;
    long long Ntot, Etot;
};

// ACT_DSWEEP: a sweep batch evaluated by the dense kernels (engine, C <= 64);
// the union kernels only apply its decisions.
enum { ACT_NONE = 0, ACT_SWEEP = 1, ACT_MERGE = 2, ACT_COMPACT = 3, ACT_DSWEEP = 4 };

#define SBP_LEAF_MAX 256
#define SBP_DENSE_MAX_C_DEV 64

// device image of the public sweep statistics record
struct sbp_sweep_stats_dev {
    long long proposals, self_proposals, accepted, near_ties;
    double sum_dS_accepted, dl_after;
};
// A decision is a near tie when its margin (-beta dS + ln H) - ln u lies within
// this of zero: a differently ordered FP64 sum of the same terms could flip it.
#define SBP_NEAR_TIE 1e-9
#define SBP_MAX_DEGREE_DEV 16384

// Index of the graph owning flat item i, given per-graph start offsets.
__device__ __forceinline__ int find_graph(const int *starts, int G, int i) {
    int lo = 0, hi = G - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}
