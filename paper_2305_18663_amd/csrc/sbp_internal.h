// sbp_internal.h -- host-side declarations shared by the library's sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "sbp_device.h"

namespace sbp {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
#define SBP_HIP_CHECK(call)                                                                     \
    do {                                                                                        \
        hipError_t err_ = (call);                                                               \
        if (err_ != hipSuccess)                                                                 \
            return ::sbp::fail(-5, std::string(#call) + ": " + hipGetErrorString(err_));        \
    } while (0)
#define SBP_LAUNCH_CHECK()                                                                      \
    do {                                                                                        \
        hipError_t err_ = hipGetLastError();                                                    \
        if (err_ != hipSuccess)                                                                 \
            return ::sbp::fail(-5, std::string("kernel launch: ") + hipGetErrorString(err_));   \
    } while (0)

// ---------------------------------------------------------------- kernel timing (sbp_engine.hip)
// Records an event pair around a launch when profiling is on.
// Timing of one measured launch while profiling is on.  By default the scope
// records its events on the stream around whatever it encloses; with attach,
// it only creates them (start, stop) for the caller to hand to
// hipExtLaunchKernelGGL, which takes the kernel's own start and stop times
// without separate stream packets.
struct ProfileScope {
    int slot = -1;
    hipStream_t s;
    const char *name_ = nullptr;
    bool attach_ = false;
    hipEvent_t start = nullptr, stop = nullptr;
    ProfileScope(const char *name, hipStream_t stream, bool attach = false);
    ~ProfileScope();
};

// ---------------------------------------------------------------- bump allocator over caller memory
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    bool dry = false;  // size query only
    Arena() = default;
    Arena(void *b, size_t c) : base((char *)b), cap(c) {}
    static Arena measure() {
        Arena a;
        a.dry = true;
        a.cap = SIZE_MAX;
        return a;
    }
    template <class T>
    T *take(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
        if (bytes == 0) bytes = 256;
        T *p = dry ? nullptr : (T *)(base + used);
        used += bytes;
        return p;
    }
    bool ok() const { return used <= cap; }
};

inline int ceil_log2(uint64_t x) {
    int b = 0;
    while (b < 64 && (1ull << b) < x) ++b;
    return b;
}
inline int grid_for(long long n, int block, int max_blocks = 65535 * 16) {
    long long g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > max_blocks) g = max_blocks;
    return (int)g;
}

// ---------------------------------------------------------------- primitives (sbp_prims.hip)
// Workspace of an exclusive scan of n elements.
size_t scan_temp_bytes(long long n);
// out[i] = sum_{j<i} in[j] (int64 out); *total (device, nullable) = sum of all.
int scan_exclusive_i32(const int *in, long long *out, long long n, long long *total, void *temp, hipStream_t s);
int scan_exclusive_i64(const long long *in, long long *out, long long n, long long *total, void *temp,
                       hipStream_t s);
// Stable LSD radix sort of n keys (< 2^bits) with optional 64-bit values.
// Results end in keys/vals (ping-pong through the alt buffers).
size_t radix_temp_bytes(long long n);
int radix_sort(uint64_t *keys, uint64_t *keys_alt, uint64_t *vals, uint64_t *vals_alt, long long n, int bits,
               void *temp, hipStream_t s);
// LSD passes over bits [lo, hi) only (stable, so equal digits keep their order).
int radix_sort_bits(uint64_t *keys, uint64_t *keys_alt, uint64_t *vals, uint64_t *vals_alt, long long n, int lo,
                    int hi, void *temp, hipStream_t s);
int fill_i32(int *p, int value, long long n, hipStream_t s);
int fill_i64(long long *p, long long value, long long n, hipStream_t s);
int iota_i32(int *p, long long n, hipStream_t s);

// ---------------------------------------------------------------- union (batched) sparse blockmodel
struct SparseBM {
    int Ctot;       // blocks in the union
    long long cap;  // entry capacity (>= union edge count)
    int *rptr;      // [Ctot+1] rows of M (entries sorted by column)
    int *rcol, *rval;
    int *cptr;      // [Ctot+1] columns of M (entries sorted by row)
    int *crow, *cval;
    int *scol, *scum;  // [2 cap] rows of M + M^T in ascending column, running sums
    int *dout, *din;   // [Ctot]
    long long *nnz;    // device scalar
};

// Scratch of one union build / step (capacities: cap >= max(total edges,
// total vertices); per-graph arrays hold G entries).
struct UnionScratch {
    uint64_t *k0, *k1, *v0, *v1;  // sort buffers [cap]
    long long *s0, *s1;           // scan outputs [cap + 1]
    int *i0, *i1;                 // int scratch [cap]
    void *temp;                   // primitive temp
    double *dl_part;              // per-chunk partial sums
    double *dl;                   // per-graph DL [G]
    int *nb;                      // accepted new label per union vertex, else -1
    int *hub_scratch;             // hub_slots x hub_scratch_ints_per_slot()
    int hub_slots;
    int *mpos, *mj0, *mj1, *mm0, *mm1, *mcyc, *mlow, *mmap;  // merge application [cap]
    int *gC;                      // per-graph new block count [G]
};

int build_union_sparse(const GDev *dG, const StepMeta &m, SparseBM &bm, UnionScratch &ws, hipStream_t s);
int union_dl(const GDev *dG, const StepMeta &m, const SparseBM &bm, UnionScratch &ws, hipStream_t s);
struct SweepTraceDev {
    int *prop;
    double *dS, *lnH, *margin;
    signed char *accept;
    signed char *status;  // -1 own block proposed, 0 rejected, 1 accepted
};
int union_sweep(const GDev *dG, const StepMeta &m, const SparseBM &bm, UnionScratch &ws, const SweepTraceDev &tr,
                hipStream_t s);
int union_merge_scores(const GDev *dG, const StepMeta &m, const SparseBM &bm, int *partner, double *dS, double *dSl,
                       hipStream_t s);
// Merge application of the merging graphs: new labels per merge item in
// ws.mmap, new block counts in ws.gC.
int union_merge_apply(const GDev *dG, const StepMeta &m, const int *partner, const double *dSl, UnionScratch &ws,
                      hipStream_t s);
// Compaction of the compacting graphs: map in ws.mmap, counts in ws.gC.
int union_compact(const GDev *dG, const StepMeta &m, UnionScratch &ws, hipStream_t s);
// lab[v] <- map[blkstart[g] + lab[v]] for the vertex items of vstart.
int union_relabel(const GDev *dG, int G, const int *vstart, int n_vitems, const int *blkstart, const int *map,
                  hipStream_t s);
// Fill the C x C lookup tables (GDev.mdense) of the graphs that have one
// (n_list of the nG graphs) from the union blockmodel.
int union_lookup_tables(const GDev *dG, int nG, int n_list, const SparseBM &bm, hipStream_t s);
constexpr int SBP_TABLE_MAX_C = 2048;  // block counts that get a lookup table
// The union blockmodel counted into the graphs' tables (every graph of the
// step has GDev.mdense; list [n_list] = all graph indices): the same arrays as
// build_union_sparse, which the tables then also serve as lookups.
int build_union_from_tables(const GDev *dG, const StepMeta &m, SparseBM &bm, UnionScratch &ws,
                            const int *list, int n_list, hipStream_t s);
// Divide-and-conquer combination choice (best[c2] for every community C1 + c2).
int union_combine_choice(const SparseBM &bm, int C1, int C2, int *best, hipStream_t s);
// Sparse blockmodel of one graph for C labels, built in a single-graph workspace.
size_t sparse_one_bytes(int n, int e);
int build_sparse_one(const GDev &d, void *ws, size_t ws_bytes, SparseBM &out, hipStream_t s);
size_t hub_scratch_ints_per_slot();
int graph_from_edges(int n, long long e, const int *src, const int *dst, int *out_ptr, int *out_idx, int *in_ptr,
                     int *in_idx, UnionScratch &ws, long long *count, int *flag, hipStream_t s);
int dl_chunks_of(int e, int C);

// ---------------------------------------------------------------- dense tier (sbp_dense.hip)
struct DenseBM {
    int C;
    int *M;           // [C*C]
    double *fM;       // [C*C] f(M_ab) = M_ab ln M_ab of the current M
    int *dout, *din;  // [C]
    double *dl;       // [1]
    double *ftab;     // [ftab_max + 1] f(x) = x ln x for every count 0 <= x <= e
    unsigned ftab_max;  // = max(e, 0): no entry of M and no block degree exceeds e
    // Block of the far end of every edge end, one byte each, in CSR order:
    // nl[0, e) for the out-ends, nl[nl_in, nl_in + e) for the in-ends;
    // 0xff marks a self-loop (its far end is the vertex itself).
    unsigned char *nl;
    long long nl_in;
    // Vertex ranges of the single-batch update: [0] = the grid they were made
    // for (0: none), [1 + w] = first vertex of workgroup w, [1 + grid] = n.
    int *bounds;
    // The other end of the same edge for every edge end: mir_o[p] is the
    // in-end position of out-end p, mir_i[q] the out-end position of in-end q
    // (a bijection on each multi-edge).  flags[0] = 1 when every mirror was
    // verified at build; flags[1] = 1 when the last single-batch update left
    // the end bytes of the moved vertices' neighbours to the final kernel.
    int *mir_o, *mir_i;
    int *flags;
};
#define SBP_DENSE_BOUNDS 1026
struct DenseScratch {
    int *delta;             // [C*C] change of M of one batch (kept zero between batches)
    int nwg;                // workgroups of the evaluation grid
    int *nb;                // [n] accepted new label, else -1 (single batch: bytes, 0xff = stays)
    long long *stats_part;  // [nwg + 1][4]; slot nwg: the hybrid sweep's sequential pass
    double *sum_part;       // [nwg + 1]
    const int *hubrank;     // nullable: > 0 for the vertices the sequential pass moved
    int hub_slot = -1;      // the sequential pass's statistics slot (first batch), or -1
};
// Hybrid sweep, sequential part, dense tier: the n_hubs vertices of highest
// degree move one at a time (order, hubrank and the sort buffers are scratch).
// Scratch of the sequential pass: sort keys [n] (k0, k1), radix temp, and
// per hub (nh <= SBP_HUBS_MAX) the vertex, out | in << 16 end counts and end
// offsets [nh + 1]; per hub edge end (at most 2e) a neighbour code and a
// mirror position; hubrank [n].
struct HubScratch {
    uint64_t *k0, *k1;
    void *temp;
    int *order, *kk, *hoff, *codes, *mpos, *hubrank;
};
int dense_hub_pass(const GDev &g, DenseBM &bm, DenseScratch &ws, int n_hubs, const HubScratch &h,
                   const SweepTraceDev &tr, hipStream_t s);
constexpr int SBP_HUBS_MAX = 4096;
int dense_build(const GDev &g, DenseBM &bm, int *delta, hipStream_t s);
int dense_sweep_batch(const GDev &g, DenseBM &bm, DenseScratch &ws, const SweepTraceDev &tr,
                      sbp_sweep_stats_dev *stats, hipStream_t s);
int dense_merge_scores(const GDev &g, const DenseBM &bm, int *partner, double *dS, double *dSl, hipStream_t s);
// Recompute the per-end block bytes from the labels (after a sweep of several
// batches, whose moves update M but not the bytes).
int dense_refresh_ends(const GDev &g, DenseBM &bm, hipStream_t s);
int dense_workgroups();
int dense_tune(const char *key, long long value);
// One graph's sweep batch on the engine's dense path: the graph (labels, CSR,
// C, seed, sweep index, batch, eps, beta; boff = its first union block), its
// dense slot (M and f(M) [C*C], degrees [C]) and its decisions [n] (ints,
// -1 = stays).
struct DenseSweepJob {
    GDev g;
    int *M;
    double *fM;
    int *dout, *din;
    int *nb;
};
size_t dense_multi_scratch_bytes(int max_graphs);
void fill_ftab(double *tab, unsigned n_max, hipStream_t s);
int dense_multi_sweep(const std::vector<DenseSweepJob> &jobs, const SparseBM &bm, const double *ftab,
                      unsigned ftab_max, void *scratch, int max_graphs, hipStream_t s);

}  // namespace sbp
