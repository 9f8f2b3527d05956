// sbp_dense.hip -- dense blockmodel tier for C <= 64 blocks (gfx950).
//
// With at most 64 blocks M (C x C int32, Sec. II-A), f(M) and the block
// degrees live in global memory and are staged in LDS by every workgroup of a
// sweep; the proposal's running sums of e_t. = M_t. + M_.t come from the
// staged M.  The blockmodel also keeps, for every edge end, the block of its
// far end as one byte (C <= 64 fits), in CSR order, so that a sweep reads its
// neighbour blocks as a contiguous stream instead of gathering a label per
// end.  A single-batch sweep is three launches:
//   eval   -- persistent grid over chunks of vertices: neighbour-block
//             histograms in LDS from the end bytes, Philox proposal, DL change
//             over the changed entries of M and the block degrees (Eq. 1-2),
//             Hastings term, accept test (Alg. 2), all against the snapshot
//             taken at the start of the sweep; writes the accepted block per
//             vertex;
//   update -- walks every edge end once: gathers the far end's decision,
//             rewrites the end byte, and for every out-edge with a moved
//             endpoint moves one count of M from (old, old) to (new, new)
//             (adjacent vertices that move together change their shared
//             edge's entry once, which is why the per-vertex change vectors
//             used for scoring cannot simply be added up); applies the labels.
//             Workgroup deltas of M in LDS are flushed with integer atomics,
//             so M does not depend on thread order.  When few vertices moved
//             it walks only their edges instead;
//   final  -- M += delta, f(M), block degrees, DL (one workgroup, fixed
//             order), sweep totals; its other workgroups write the moved
//             vertices' new blocks into the end bytes that point at them
//             after a move-driven update.
// A sweep of several batches evaluates each batch against the labels (the
// bytes would go stale within the sweep), walks only the moved vertices for
// the delta, and recomputes the end bytes once at the end.
#include <string.h>

#include <hip/hip_ext.h>

#include "sbp_internal.h"

namespace sbp {

namespace {

constexpr int DC = SBP_DENSE_MAX_C_DEV;

__device__ __forceinline__ double model_terms_d(double E, double N, double C) {
    const double c2 = C * C;
    return xlogx(E + c2) - xlogx(E) - xlogx(c2) + N * log(C);
}

__global__ void k_zero(int *p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// M_ab += number of edges from block a to block b, per-workgroup LDS histogram
__global__ void __launch_bounds__(256) k_dense_hist(GDev g, int *__restrict__ M) {
    __shared__ int H[DC * DC];
    const int C = g.C, CC = C * C;
    for (int i = threadIdx.x; i < CC; i += blockDim.x) H[i] = 0;
    __syncthreads();
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += gridDim.x * blockDim.x) {
        const int a = g.lab[v] * C;
        const int j1 = g.out_ptr[v + 1];
        for (int j = g.out_ptr[v]; j < j1; ++j) atomicAdd(&H[a + g.lab[g.out_idx[j]]], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < CC; i += blockDim.x)
        if (H[i]) atomicAdd(&M[i], H[i]);
}

// Block of the far end of every edge end (0xff for a self-loop), wave per
// vertex.
__global__ void __launch_bounds__(256) k_dense_ends(GDev g, DenseBM bm) {
    const int lane = threadIdx.x & 63;
    unsigned char *nlo = bm.nl, *nli = bm.nl + bm.nl_in;
    for (int v = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; v < g.n; v += (gridDim.x * blockDim.x) >> 6) {
        const int o1 = g.out_ptr[v + 1], i1 = g.in_ptr[v + 1];
        for (int j = g.out_ptr[v] + lane; j < o1; j += 64) {
            const int u = g.out_idx[j];
            nlo[j] = u == v ? 0xffu : (unsigned char)g.lab[u];
        }
        for (int j = g.in_ptr[v] + lane; j < i1; j += 64) {
            const int u = g.in_idx[j];
            nli[j] = u == v ? 0xffu : (unsigned char)g.lab[u];
        }
    }
}

// Mirror positions of every edge end, a wave per vertex v: out-end p to u is
// the r-th copy of u in v's ascending out-list and its in-end the r-th copy of
// v in u's ascending in-list.  Every match is checked (lists ascending, the
// copy present); any failure clears flags[0], and so does an in-end left
// without a mirror (k_dense_mirror_check), so the mirrors are only used when
// they form a bijection of the edges.
__global__ void __launch_bounds__(256) k_dense_mirror(GDev g, DenseBM bm) {
    const int lane = threadIdx.x & 63;
    for (int v = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; v < g.n; v += (gridDim.x * blockDim.x) >> 6) {
        const int o0 = g.out_ptr[v], o1 = g.out_ptr[v + 1];
        for (int p = o0 + lane; p < o1; p += 64) {
            const int u = g.out_idx[p];
            bool ok = p == o0 || g.out_idx[p - 1] <= u;
            int lo = o0, hi = p;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (g.out_idx[mid] < u) lo = mid + 1; else hi = mid;
            }
            const int i0 = g.in_ptr[u], i1 = g.in_ptr[u + 1];
            int l2 = i0, h2 = i1;
            while (l2 < h2) {
                const int mid = (l2 + h2) >> 1;
                if (g.in_idx[mid] < v) l2 = mid + 1; else h2 = mid;
            }
            const int q = l2 + (p - lo);
            ok = ok && q < i1 && g.in_idx[q] == v;
            if (ok) {
                bm.mir_o[p] = q;
                bm.mir_i[q] = p;
            } else {
                bm.mir_o[p] = -1;
                bm.flags[0] = 0;
            }
        }
        const int j0 = g.in_ptr[v], j1 = g.in_ptr[v + 1];
        for (int q = j0 + 1 + lane; q < j1; q += 64)
            if (g.in_idx[q - 1] > g.in_idx[q]) bm.flags[0] = 0;
    }
}
__global__ void k_set_flags(int *flags) {
    flags[0] = 1;
    flags[1] = 0;
}
__global__ void k_dense_mirror_check(const DenseBM bm, int e) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < e; q += gridDim.x * blockDim.x)
        if (bm.mir_i[q] < 0) bm.flags[0] = 0;
}

// Moved-vertex part of the end-byte update (workgroups 1.. of the final
// kernel after a move-driven update): every moved vertex writes its new block
// into the mirror of each of its edge ends, i.e. into the end bytes that point
// at it.  Self-loop ends (0xff) never change.
__device__ void mirror_bytes(const GDev &g, const DenseBM &bm, const unsigned char *__restrict__ nb, int wg, int nwg) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    unsigned char *nlo = bm.nl, *nli = bm.nl + bm.nl_in;
    const int v0 = (int)((long long)g.n * wg / nwg), v1 = (int)((long long)g.n * (wg + 1) / nwg);
    const int elast = max(g.e - 1, 0);
    for (int tb = v0 + wv * 64; tb < v1; tb += nw * 64) {
        const int v = tb + lane;
        const unsigned x = v < v1 ? nb[v] : 0xffu;
        // every moved lane's end ranges in one round trip
        const int vc = min(v, g.n - 1);
        const int lo0 = g.out_ptr[vc], lo1 = g.out_ptr[vc + 1], li0 = g.in_ptr[vc], li1 = g.in_ptr[vc + 1];
        for (uint64_t todo = __ballot(x != 0xffu); todo; todo &= todo - 1) {
            const int l = __builtin_ctzll(todo);
            const unsigned char xn = (unsigned char)__shfl((int)x, l, 64);
            const int o0 = __shfl(lo0, l, 64), ko = __shfl(lo1, l, 64) - o0;
            const int i0 = __shfl(li0, l, 64), ki = __shfl(li1, l, 64) - i0;
            // out-end j and in-end j together, loads unconditional (positions clamped)
            for (int j = lane; j < max(ko, ki); j += 64) {
                const int p = min(o0 + j, elast), q = min(i0 + j, elast);
                const int mq = bm.mir_o[p], mp = bm.mir_i[q];
                const unsigned bo = nlo[p], bi = nli[q];
                if (j < ko && bo != 0xffu && (unsigned)mq < (unsigned)g.e) nli[mq] = xn;
                if (j < ki && bi != 0xffu && (unsigned)mp < (unsigned)g.e) nlo[mp] = xn;
            }
        }
    }
}

// Vertex ranges of equal cost for a grid of G workgroups: cost(v) is the
// number of edge ends of vertices below v plus wV per vertex below v, which is
// monotone in v, so range w starts at the first v with cost(v) >= w/G of the
// total.  out[0] = G, out[1 + w] for w = 0..G (out[1] = 0, out[1 + G] = n).
__global__ void k_dense_bounds(GDev g, int G, int wV, int *__restrict__ out) {
    if (G <= 0) {  // no ranges: the kernels deal chunks round robin
        if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
        return;
    }
    const long long total = (long long)g.out_ptr[g.n] + g.in_ptr[g.n] + (long long)wV * g.n;
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w <= G; w += gridDim.x * blockDim.x) {
        const long long target = total * w / G;
        int lo = 0, hi = g.n;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const long long c = (long long)g.out_ptr[mid] + g.in_ptr[mid] + (long long)wV * mid;
            if (c >= target) hi = mid; else lo = mid + 1;
        }
        out[1 + w] = lo;
        if (w == 0) out[0] = G;
    }
}

// f(x) = x ln x for every count 0 <= x <= e (no entry of M and no block degree
// can exceed the number of edges), computed on the device with the same xlogx
// as a direct evaluation, so a lookup returns the very value a direct
// evaluation would.  Lookups clamp the index, so an inconsistent state reads a
// wrong value instead of out of bounds.
__global__ void k_ftab(double *__restrict__ tab, unsigned n_max) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i <= (long long)n_max;
         i += (long long)gridDim.x * blockDim.x)
        tab[i] = xlogx((double)i);
}
__device__ __forceinline__ double fx(const double *__restrict__ tab, unsigned n_max, int x) {
    return tab[min((unsigned)x, n_max)];
}

// M += delta (delta cleared), f(M), block degrees and DL; sweep totals.  One
// workgroup, a thread per entry of M: the statistics partials, M and the delta
// are read together, degrees are exact LDS integer sums, and the DL sum is
// taken in a fixed order.
constexpr int FIN_T = 512;
__global__ void __launch_bounds__(FIN_T) k_dense_final(GDev g, DenseBM bm, int *__restrict__ delta,
                                                      const long long *__restrict__ stats_part,
                                                      const double *__restrict__ sum_part, int nwg,
                                                      sbp_sweep_stats_dev *__restrict__ stats,
                                                      const unsigned char *__restrict__ nbm, int extra) {
    if (blockIdx.x > 0) {  // end bytes of the moved vertices' neighbours, after a move-driven update
        if (nbm && bm.flags[1]) mirror_bytes(g, bm, nbm, blockIdx.x - 1, gridDim.x - 1);
        return;
    }
    __shared__ int so[DC], si[DC];
    __shared__ double wred[FIN_T / 64], sred[FIN_T / 64];
    __shared__ long long lred[4][FIN_T / 64];
    const int C = g.C, CC = C * C, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const double *tab = bm.ftab;
    const unsigned fmax = bm.ftab_max;
    long long a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    double sd = 0.0;
    if (stats) {
        for (int w = tid; w < nwg; w += FIN_T) {
            a0 += stats_part[4 * w + 0];
            a1 += stats_part[4 * w + 1];
            a2 += stats_part[4 * w + 2];
            a3 += stats_part[4 * w + 3];
            sd += sum_part[w];
        }
        if (extra >= 0 && tid == 0) {  // the sequential pass's totals
            a0 += stats_part[4 * extra + 0];
            a1 += stats_part[4 * extra + 1];
            a2 += stats_part[4 * extra + 2];
            a3 += stats_part[4 * extra + 3];
            sd += sum_part[extra];
        }
    }
    if (tid < C) {
        so[tid] = 0;
        si[tid] = 0;
    }
    __syncthreads();
    // L = sum f(M) - sum f(dout) - sum f(din)
    double acc = 0.0;
    for (int i = tid; i < CC; i += FIN_T) {
        const int d = delta[i];
        int m = bm.M[i];
        if (d) {
            m += d;
            bm.M[i] = m;
            delta[i] = 0;
        }
        const double f = fx(tab, fmax, m);
        bm.fM[i] = f;
        acc += f;
        const int row = i / C;
        atomicAdd(&so[row], m);
        atomicAdd(&si[i - row * C], m);
    }
    __syncthreads();
    if (tid < C) {
        const int o = so[tid], n = si[tid];
        bm.dout[tid] = o;
        bm.din[tid] = n;
        acc -= fx(tab, fmax, o) + fx(tab, fmax, n);
    }
    acc = wave_sum(acc);
    a0 = wave_sum_i64(a0);
    a1 = wave_sum_i64(a1);
    a2 = wave_sum_i64(a2);
    a3 = wave_sum_i64(a3);
    sd = wave_sum(sd);
    if (lane == 0) {
        wred[wv] = acc;
        lred[0][wv] = a0;
        lred[1][wv] = a1;
        lred[2][wv] = a2;
        lred[3][wv] = a3;
        sred[wv] = sd;
    }
    __syncthreads();
    if (tid == 0) {
        double L = 0.0, sdt = 0.0;
        long long p = 0, sp = 0, ac = 0, ti = 0;
        for (int w = 0; w < FIN_T / 64; ++w) {
            L += wred[w];
            p += lred[0][w];
            sp += lred[1][w];
            ac += lred[2][w];
            ti += lred[3][w];
            sdt += sred[w];
        }
        const double dl = model_terms_d((double)g.e, (double)g.n, (double)C) - L;
        bm.dl[0] = dl;
        if (stats) {  // the first batch of a sweep starts the totals
            const bool first = g.batch == 0;
            stats->proposals = (first ? 0 : stats->proposals) + p;
            stats->self_proposals = (first ? 0 : stats->self_proposals) + sp;
            stats->accepted = (first ? 0 : stats->accepted) + ac;
            stats->near_ties = (first ? 0 : stats->near_ties) + ti;
            stats->sum_dS_accepted = (first ? 0.0 : stats->sum_dS_accepted) + sdt;
            stats->dl_after = dl;
        }
        if (g.sweep_dev && g.action == ACT_SWEEP && g.batch == g.n_batches - 1) *g.sweep_dev += 1u;
    }
}

// Inclusive prefix sum over the GS = 4 or 8 lanes of a scoring group (gl =
// lane in the group): row shifts, with the lanes whose source lies in the
// group before left out.
template <int GS>
__device__ __forceinline__ int grp_scan(int x, int gl) {
    int y = __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    if (gl >= 1) x += y;
    y = __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    if (gl >= 2) x += y;
    if (GS >= 8) {
        y = __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
        if (gl >= 4) x += y;
    }
    return x;
}

constexpr int EVAL_T = 256;      // threads per workgroup
constexpr int SEG = 8;           // consecutive edge ends per thread in the histogram phase
constexpr int LDS_CU = 160 * 1024;

// Arguments of the evaluation kernel: only what it reads, so that the
// uniform values fit the scalar registers.
struct EvalArgs {
    const int *out_ptr, *in_ptr, *out_idx, *in_idx;
    const int *lab;
    const int *M, *dout, *din;
    const double *fM, *ftab;
    const unsigned char *nlo, *nli;
    const int *hubrank;  // nullable: > 0 for the vertices the sequential pass already moved
    void *nb;
    long long *stats_part;
    double *sum_part;
    unsigned long long seed;
    double beta;
    unsigned ftab_max, sweep;
    int n, C, batch, n_batches, eps, voff;
    const unsigned *sweep_dev;  // nullable: the sweep index in device memory
};

// Static LDS of the evaluation kernel for up to CM blocks: every array sits at
// a fixed offset.  Rows of M and f(M) are RS = CM + 1 apart (an odd number of
// words), so a column walk by 16 lanes hits 16 different banks; histogram
// rows are CM apart.
template <int CM>
struct EvalLds {
    // lanes per vertex in the scoring phase: four up to 48 blocks (sixteen
    // vertices per wave), eight (half a DPP row) beyond
    static constexpr int GS = CM > 48 ? 8 : 4;
    static constexpr int NG = EVAL_T / GS;         // scoring groups per workgroup
    static constexpr int CH = CM > 48 ? 32 : 64;  // vertices per chunk
    // waves a SIMD can hold with this LDS (three workgroups a CU up to 48
    // blocks, two beyond): the register budget follows from it
    static constexpr int WAVES = CM > 48 ? 2 : 3;
    static constexpr int RS = CM + 1;
    double fM[CM * RS];
    double fdo[CM], fdi[CM], inv[CM];
    uint64_t W[4][CH];  // Philox words 0-3 of the chunk's vertices
    long long wst[4 * (EVAL_T / 64)];
    double wsd[EVAL_T / 64];
    int Ms[CM * RS];
    int dsum[CM], dos[CM], dis[CM];
    unsigned H[CH * CM];  // out-ends in the low 16 bits, in-ends in the high 16 bits
    int v[CH], r[CH], op[CH + 1], kout[CH], ip[CH + 1], kin[CH], pre[CH + 1], ell[CH], t0[CH], j0[CH];
    unsigned char items[NG][CM + 1];  // the last byte takes the writes of unlisted blocks
};
template <int CM>
constexpr int eval_chunk() { return EvalLds<CM>::CH; }
template <int CM>
constexpr int eval_wgs_per_cu() {
    return (int)(LDS_CU / sizeof(EvalLds<CM>)) < 4 ? (int)(LDS_CU / sizeof(EvalLds<CM>)) : 4;
}

// Sweep batch evaluation against the snapshot M.  A workgroup takes CH batch
// vertices at a time:
//  (0) their pointers, labels and end prefix (wave 0), their Philox words and
//      end draws (wave 1) and empty histogram rows (waves 2-3), together;
//  (A) every edge end of the chunk into packed per-vertex block histograms in
//      LDS: a thread takes SEG consecutive ends of the chunk's flattened end
//      list, finds their owners with one search and a forward walk, issues all
//      its loads, then counts.  With ENDS the far-end blocks are the stored end
//      bytes; otherwise (one batch of several) the ids are read and the labels
//      gathered;
//  (B) a group of GS lanes (four, or eight past 48 blocks) scores one vertex
//      per round: the proposal from running sums of e_t0. built on the fly
//      from M (exact integer sums, lane gl owning NQ consecutive blocks, one
//      group scan), the vertex's nonzero blocks t != r, s compacted into a
//      list in block order, then for every listed block the four changed
//      entries of M -- f of the old values from LDS, f of the new values
//      gathered from the table, a batch of gathers (with the 2x2 corner and
//      the block degrees) in flight together -- the Hastings terms, group
//      sums on DPP and the three logs of the wave's 64 / GS vertices in one
//      evaluation.
// The decision goes to nb: with ENDS one byte per vertex (0xff = stays),
// otherwise an int (-1 = stays).  TRACE adds the per-vertex record.
//
// The chunks a workgroup takes come from a chunk source: the strided split of
// one graph's chunks over the grid (StridedChunks), or runs of consecutive
// chunks pulled from a graph's work queue (QueueChunks).
struct StridedChunks {
    int cur, stride, n;
    __device__ __forceinline__ int first(int nchunks) {
        n = nchunks;
        return cur < n ? cur : -1;
    }
    __device__ __forceinline__ int next() {
        cur += stride;
        return cur < n ? cur : -1;
    }
};
// Runs of `run_len` consecutive chunks; `cur` starts as the first chunk of a
// run already taken.  A new run is pulled with one atomic by thread 0 and one
// barrier; the pulled index is read before the next barrier of the chunk loop,
// so the next pull cannot overwrite it early.
struct QueueChunks {
    int *ctr;      // the graph's queue: next run index
    int *pull;     // LDS word for the pulled index
    int run_len, cur, end, n;
    __device__ __forceinline__ int first(int nchunks) {
        n = nchunks;
        end = min(cur + run_len, n);
        return cur < n ? cur : -1;
    }
    __device__ __forceinline__ int next() {
        if (++cur < end) return cur;
        if (threadIdx.x == 0) *pull = atomicAdd(ctr, 1);
        __syncthreads();
        cur = __builtin_amdgcn_readfirstlane(*pull) * run_len;
        end = min(cur + run_len, n);
        return cur < n ? cur : -1;
    }
};

template <bool ENDS, bool TRACE, int CM, class Chunks>
__device__ __forceinline__ void eval_body(EvalLds<CM> &L, const EvalArgs &a, const SweepTraceDev &tr, Chunks src) {
    using Lds = EvalLds<CM>;
    constexpr int CH = Lds::CH;
    constexpr int RS = Lds::RS;
    constexpr int GS = Lds::GS, NG = Lds::NG;
    constexpr unsigned GMASK = (1u << GS) - 1u;
    constexpr int NQ = CM / GS;  // blocks per lane in the scoring phase
    constexpr int BQ = NQ < 2 ? NQ : 2;  // slots per batch of table gathers
    static_assert(CH % NG == 0, "every group scores the same number of vertices per chunk");
    const double *__restrict__ tab = a.ftab;
    const unsigned fmax = a.ftab_max;
    const int C = a.C;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int grp = tid / GS, gl = tid % GS, wgrp = lane / GS;  // group in workgroup / in wave
    const double eps = (double)a.eps, epsC = (double)a.eps * (double)C;
    const long long eC = (long long)a.eps * C;
    for (int i = tid; i < C * C; i += EVAL_T) {
        const int x = i / C, y = i - x * C;
        L.Ms[x * RS + y] = a.M[i];
        L.fM[x * RS + y] = a.fM[i];
    }
    if (tid < C) {
        const int o = a.dout[tid], n = a.din[tid];
        L.dos[tid] = o;
        L.dis[tid] = n;
        L.dsum[tid] = o + n;
        L.fdo[tid] = fx(tab, fmax, o);
        L.fdi[tid] = fx(tab, fmax, n);
        L.inv[tid] = 1.0 / ((double)(o + n) + epsC);
    }
    long long n_prop = 0, n_self = 0, n_acc = 0;
    int n_tie = 0;
    double s_dS = 0.0;
    const unsigned sweep = a.sweep_dev ? *a.sweep_dev : a.sweep;
    const int nbc = (a.n - a.batch + a.n_batches - 1) / a.n_batches;
    const int nchunks = (nbc + CH - 1) / CH;
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    for (int chunk = src.first(nchunks); chunk >= 0; chunk = src.next()) {
        const int base = chunk * CH;
        const int nv = min(CH, nbc - base);
        __syncthreads();  // previous chunk done with the LDS
        // (0) three waves in parallel: the chunk's vertex data (wave 0), the
        // Philox words (wave 1), empty histograms (the rest)
        if (wv == 0) {
            int k = 0;
            if (lane < nv) {
                const int v = a.batch + (base + lane) * a.n_batches;
                const int op = a.out_ptr[v], ko = a.out_ptr[v + 1] - op;
                const int ip = a.in_ptr[v], ki = a.in_ptr[v + 1] - ip;
                L.v[lane] = v;
                L.r[lane] = a.lab[v];
                L.op[lane] = op;
                L.kout[lane] = ko;
                L.ip[lane] = ip;
                L.kin[lane] = ki;
                L.ell[lane] = 0;
                k = ko + ki;
                if (lane == nv - 1) {  // ends of the chunk's ranges (consecutive vertices)
                    L.op[nv] = op + ko;
                    L.ip[nv] = ip + ki;
                }
            }
            // exclusive prefix of the edge-end counts
            int x = k;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o, SBP_WAVE);
                if (lane >= o) x += y;
            }
            if (lane < CH) L.pre[lane + 1] = x;
            if (lane == 0) L.pre[0] = 0;
        } else if (wv == 1) {
            // blocks (v, sweep, 0, 0) and (v, sweep, 1, 0): words W0, W1 and W2, W3
            for (int i = lane; i < 2 * CH; i += 64) {
                const int vi = i % CH, blk = i / CH;
                if (vi < nv) {
                    const int v = a.batch + (base + vi) * a.n_batches;
                    // the degree for the end draw j0 (the same words wave 0 reads)
                    const int k = blk ? 0 : a.out_ptr[v + 1] - a.out_ptr[v] + a.in_ptr[v + 1] - a.in_ptr[v];
                    uint32_t o[4];
                    philox_block((uint32_t)v, sweep, (uint32_t)blk, 0u, k0, k1, o);
                    const uint64_t Wa = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
                    L.W[2 * blk][vi] = Wa;
                    L.W[2 * blk + 1][vi] = (uint64_t)o[2] | ((uint64_t)o[3] << 32);
                    if (!blk) L.j0[vi] = k > 0 ? (int)draw_idx(Wa, (uint64_t)k) : -1;
                }
            }
        } else {
            for (int i = tid - 128; i < CH * CM; i += EVAL_T - 128) L.H[i] = 0;
        }
        __syncthreads();
        if constexpr (ENDS) {
            // (A) histograms from the end bytes: the chunk's vertices are
            // consecutive, so its out-end bytes form one range and its in-end
            // bytes another; a thread takes an 8-aligned block of a range
            // (one 8-byte load; the byte arrays are padded), finds the owner of
            // its first position and walks forward
            const int o0 = L.op[0], o1 = L.op[nv], i0 = L.ip[0], i1 = L.ip[nv];
            const int bo0 = o0 >> 3, nbo = o1 > o0 ? ((o1 + 7) >> 3) - bo0 : 0;
            const int bi0 = i0 >> 3, nbi = i1 > i0 ? ((i1 + 7) >> 3) - bi0 : 0;
            for (int rr = tid; rr < nbo + nbi; rr += EVAL_T) {
                const bool out = rr < nbo;
                const int p0 = (out ? bo0 + rr : bi0 + (rr - nbo)) * 8;
                const int lo = out ? o0 : i0, hi = out ? o1 : i1;
                const uint2 bw = *(const uint2 *)((out ? a.nlo : a.nli) + p0);
                const int *P = out ? L.op : L.ip;
                const int pf = max(lo, p0);
                int l = 0, h = nv - 1;  // owner of pf: last vertex whose range starts at or before it
                while (l < h) {
                    const int mid = (l + h + 1) >> 1;
                    if (P[mid] <= pf) l = mid; else h = mid - 1;
                }
                int w = l, beg = P[l], nxt = P[l + 1];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int p = p0 + q;
                    if (p < lo || p >= hi) continue;
                    while (p >= nxt) {
                        ++w;
                        beg = nxt;
                        nxt = P[w + 1];
                    }
                    const unsigned b = ((q < 4 ? bw.x : bw.y) >> (8 * (q & 3))) & 0xffu;
                    const int j = out ? p - beg : L.kout[w] + (p - beg);
                    int tt;
                    if (b == 0xffu) {  // self-loop end
                        tt = L.r[w];
                        if (out) atomicAdd(&L.ell[w], 1);
                    } else {
                        tt = (int)b;
                        atomicAdd(&L.H[w * CM + tt], out ? 1u : 65536u);
                    }
                    if (j == L.j0[w]) L.t0[w] = tt;
                }
            }
        } else {
            // (A) histograms: end f of the chunk is end f - pre[w] of its owner w,
            // out-ends before in-ends
            const int total = L.pre[nv];
            for (int f0 = tid * SEG; f0 < total; f0 += EVAL_T * SEG) {
                int lo = 0, hi = nv - 1;  // owner of f0: last vertex with pre <= f0
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (L.pre[mid] <= f0) lo = mid; else hi = mid - 1;
                }
                int w = lo, beg = L.pre[lo], nxt = L.pre[lo + 1];
                int wko = L.kout[lo], wop = L.op[lo], wip = L.ip[lo];
                int wq[SEG], jq[SEG], pq[SEG];
                unsigned outm = 0;
#pragma unroll
                for (int q = 0; q < SEG; ++q) {
                    const int f = f0 + q;
                    if (f < total) {
                        while (f >= nxt) {
                            ++w;
                            beg = nxt;
                            nxt = L.pre[w + 1];
                            wko = L.kout[w];
                            wop = L.op[w];
                            wip = L.ip[w];
                        }
                    }
                    const int j = f - beg;
                    const bool out = j < wko;
                    wq[q] = f < total ? w : -1;
                    jq[q] = j;
                    pq[q] = out ? wop + j : wip + (j - wko);
                    outm |= (out ? 1u : 0u) << q;
                }
                unsigned b[SEG];
                if constexpr (ENDS) {
#pragma unroll
                    for (int q = 0; q < SEG; ++q)
                        b[q] = wq[q] >= 0 ? ((outm >> q) & 1u ? a.nlo[pq[q]] : a.nli[pq[q]]) : 0xffu;
                } else {
                    int u[SEG];
#pragma unroll
                    for (int q = 0; q < SEG; ++q)
                        u[q] = wq[q] >= 0 ? ((outm >> q) & 1u ? a.out_idx[pq[q]] : a.in_idx[pq[q]]) : 0;
#pragma unroll
                    for (int q = 0; q < SEG; ++q)
                        b[q] = (wq[q] >= 0 && u[q] != L.v[wq[q]]) ? (unsigned)a.lab[u[q]] : 0xffu;
                }
#pragma unroll
                for (int q = 0; q < SEG; ++q) {
                    if (wq[q] < 0) break;
                    const int ww = wq[q];
                    const bool out = (outm >> q) & 1u;
                    int tt;
                    if (b[q] == 0xffu) {  // self-loop end
                        tt = L.r[ww];
                        if (out) atomicAdd(&L.ell[ww], 1);
                    } else {
                        tt = (int)b[q];
                        atomicAdd(&L.H[ww * CM + tt], out ? 1u : 65536u);
                    }
                    if (jq[q] == L.j0[ww]) L.t0[ww] = tt;
                }
            }
        }
        __syncthreads();
        // (B) scoring, one vertex per group per round; every group runs the
        // same number of rounds, so DPP and ballots see whole groups.  The
        // round is written without branches: every LDS read is issued whatever
        // the conditions (all indices stay inside the arrays) and the
        // conditions select among the values, so the reads of a step are in
        // flight together instead of one waited-for read per condition.
        for (int vi = grp; vi < CH; vi += NG) {
            const bool valid = vi < nv;
            const int v_ = L.v[vi], r_ = L.r[vi], ko_ = L.kout[vi], ki_ = L.kin[vi];
            const int ell_ = L.ell[vi], t0_ = L.t0[vi];
            const uint64_t W1 = L.W[1][vi], W2 = L.W[2][vi], W3 = L.W[3][vi];
            const int v = valid ? v_ : 0, r = valid ? r_ : 0;
            const int kout = valid ? ko_ : 0, kin = valid ? ki_ : 0, ell = valid ? ell_ : 0;
            const int k = kout + kin;
            const int t0 = k > 0 ? t0_ : 0;
            const unsigned *Hv = L.H + vi * CM;
            // proposal: a uniform block, or the first block b whose running
            // sum of e_t0,b' = M_t0,b' + M_b',t0 over b' <= b exceeds x; lane
            // gl holds the blocks gl NQ .. gl NQ + NQ - 1
            const int b0 = gl * NQ;
            int s;
            {
                const int dt0 = L.dsum[t0];
                const long long dt = k > 0 ? (long long)dt0 : 0;
                const bool unif = (k == 0) | (draw_idx(W1, (uint64_t)(dt + eC)) < (uint64_t)eC);
                const long long x = unif ? 0 : (long long)draw_idx(W2, (uint64_t)dt);
                int ev[NQ], lsum = 0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int e0 = L.Ms[t0 * RS + b0 + q] + L.Ms[(b0 + q) * RS + t0];  // padded rows
                    ev[q] = (!unif & (b0 + q < C)) ? e0 : 0;
                    lsum += ev[q];
                }
                const int incl = grp_scan<GS>(lsum, gl);
                const unsigned m = (unsigned)(__ballot(!unif & ((long long)incl > x)) >> (wgrp * GS)) & GMASK;
                long long acc = (long long)(incl - lsum);
                int cand = C;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    acc += ev[q];
                    cand = ((cand == C) & (acc > x)) ? b0 + q : cand;
                }
                const int sp = __shfl(cand, wgrp * GS + (m ? __builtin_ctz(m) : 0), SBP_WAVE);
                s = unif ? (int)draw_idx(W2, (uint64_t)C) : (m ? sp : C);
            }
            bool hub = false;  // moved one at a time before this pass
            if (a.hubrank) {
                const int hk = a.hubrank[v];
                hub = valid & (hk > 0);
            }
            const bool act = valid & !hub & (s != r);
            if (!act) s = r;  // keeps every index below in range
            // blocks t != r, s with a neighbour: a compacted list in block
            // order (lane gl writes its blocks after those of lanes < gl; a
            // block that is not listed is written to the spare last byte)
            unsigned char *items = L.items[grp];
            int n_it;
            {
                unsigned nzm = 0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int t = b0 + q;
                    const unsigned hv = Hv[t];  // within the padded row
                    nzm |= (act & (t < C) & (t != r) & (t != s) & (hv != 0u)) ? 1u << q : 0u;
                }
                const int cnt = __builtin_popcount(nzm);
                const int incl = grp_scan<GS>(cnt, gl);
                n_it = __shfl(incl, wgrp * GS + GS - 1, SBP_WAVE);
                int pos = incl - cnt;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const bool nz = (nzm >> q) & 1u;
                    items[nz ? pos : CM] = (unsigned char)(b0 + q);
                    pos += nz ? 1 : 0;
                }
            }
            // the corner item of this lane: entries (lanes 0-3), degrees (4-7)
            const int c = gl & 3;
            const int ca = c < 2 ? r : s, cb = (c & 1) ? s : r;  // entry (ca, cb) of the corner
            const int bc = (c & 1) ? s : r;                        // block of the degree term
            const unsigned hr = Hv[r], hs = Hv[s];
            const int m_c = L.Ms[ca * RS + cb], do_c = L.dos[bc], di_c = L.dis[bc];
            const double fm_c = L.fM[ca * RS + cb], fdo_c = L.fdo[bc], fdi_c = L.fdi[bc];
            const int Mrr = L.Ms[r * RS + r], Mrs = L.Ms[r * RS + s], Msr = L.Ms[s * RS + r], Mss = L.Ms[s * RS + s];
            const int dsr_ = L.dsum[r], dss_ = L.dsum[s];
            wave_sync_lds();  // the group's list is written
            const int ko_r = (int)(hr & 0xffffu), ki_r = (int)(hr >> 16);
            const int ko_s = (int)(hs & 0xffffu), ki_s = (int)(hs >> 16);
            const int mdelta = c == 0 ? -ko_r - ki_r - ell : c == 1 ? -ko_s + ki_r : c == 2 ? ko_r - ki_s : ko_s + ki_s + ell;
            // the entry (lanes 0-3) or the degree term (lanes 4-7) of corner
            // item c; with four lanes a group, both
            const bool is_m = GS == 4 || gl < 4;
            const int cdeg = c < 2 ? do_c : di_c;
            const int ddelta = c == 0 ? -kout : c == 1 ? kout : c == 2 ? -kin : kin;
            const int c_new = is_m ? m_c + mdelta : cdeg + ddelta;
            const double c_fnew = fx(tab, fmax, act ? c_new : 0);
            const double d_fnew = GS == 4 ? fx(tab, fmax, act ? cdeg + ddelta : 0) : 0.0;
            double dL = 0.0, qf = 0.0, qr = 0.0;
            // listed blocks: four changed entries each, BQ slots per batch, a
            // batch only when a group of the wave needs it.  Within a batch no
            // branches: a slot without a block, or a count of zero, loads f(0)
            // (one line for the whole wave) and contributes an exact zero.
#pragma unroll 1
            for (int q0 = 0; q0 < NQ; q0 += BQ) {
                if (!__any(q0 * GS < n_it)) break;
                int ti[BQ];
                unsigned hq[BQ];
#pragma unroll
                for (int q = 0; q < BQ; ++q) {
                    const int i = (q0 + q) * GS + gl;
                    const int t = items[i];
                    ti[q] = i < n_it ? t : 0;
                }
#pragma unroll
                for (int q = 0; q < BQ; ++q) {
                    const unsigned h = Hv[ti[q]];
                    hq[q] = (q0 + q) * GS + gl < n_it ? h : 0u;
                }
                double fn[BQ][4];
#pragma unroll
                for (int q = 0; q < BQ; ++q) {
                    const int t = ti[q];
                    const int ko = (int)(hq[q] & 0xffffu), ki = (int)(hq[q] >> 16);
                    const int mrt = L.Ms[r * RS + t], mst = L.Ms[s * RS + t];
                    const int mtr = L.Ms[t * RS + r], mts = L.Ms[t * RS + s];
                    fn[q][0] = fx(tab, fmax, ko ? mrt - ko : 0);
                    fn[q][1] = fx(tab, fmax, ko ? mst + ko : 0);
                    fn[q][2] = fx(tab, fmax, ki ? mtr - ki : 0);
                    fn[q][3] = fx(tab, fmax, ki ? mts + ki : 0);
                    // Hastings terms while the gathers are in flight (zero for an empty slot)
                    const double kt = (double)(ko + ki), iv = L.inv[t];
                    qf += kt * (((double)(mts + mst) + eps) * iv);
                    qr += kt * (((double)(mtr - ki + mrt - ko) + eps) * iv);
                }
#pragma unroll
                for (int q = 0; q < BQ; ++q) {
                    const int t = ti[q];
                    const int ko = (int)(hq[q] & 0xffffu), ki = (int)(hq[q] >> 16);
                    const double f0 = L.fM[r * RS + t], f1 = L.fM[s * RS + t];
                    const double f2 = L.fM[t * RS + r], f3 = L.fM[t * RS + s];
                    const double d_out = (fn[q][0] - f0) + (fn[q][1] - f1);
                    const double d_in = (fn[q][2] - f2) + (fn[q][3] - f3);
                    dL += (ko ? d_out : 0.0) + (ki ? d_in : 0.0);
                }
            }
            {
                const double d_fold = c < 2 ? fdo_c : fdi_c;
                if constexpr (GS == 4) {
                    dL += act ? (c_fnew - fm_c) - (d_fnew - d_fold) : 0.0;
                } else {
                    const double c_fold = is_m ? fm_c : d_fold;
                    dL += act ? (is_m ? 1.0 : -1.0) * (c_fnew - c_fold) : 0.0;
                }
            }
            // Hastings terms of t = r and t = s (lanes 0-3): before, after;
            // every lane evaluates, lanes 4-7 and idle vertices add zero
            {
                const int drr = -ko_r - ki_r - ell, drs = -ko_s + ki_r, dsr = ko_r - ki_s;
                const int kk = c == 0 ? ko_r + ki_r + 2 * ell : c == 1 ? ko_s + ki_s : c == 2 ? ko_r + ki_r : ko_s + ki_s + 2 * ell;
                const int num = c == 0 ? Mrs + Msr : c == 1 ? 2 * Mss : c == 2 ? 2 * (Mrr + drr) : Msr + dsr + Mrs + drs;
                const int den = c == 0 ? dsr_ : c == 1 ? dss_ : c == 2 ? dsr_ - k : dss_ + k;
                const double term = (double)kk * (((double)num + eps) / ((double)den + epsC));
                const bool use = act & is_m & (kk != 0);
                qf += (use & (c < 2)) ? term : 0.0;
                qr += (use & (c >= 2)) ? term : 0.0;
            }
            dL = grp_sum<GS>(dL);
            qf = grp_sum<GS>(qf);
            qr = grp_sum<GS>(qr);
            // the three logs of the wave's 64/GS vertices in one evaluation
            double lg;
            {
                const double u = draw_unit(W3);
                const int q = lane / 3, m = lane % 3;
                const int src = (q < 64 / GS ? q : 0) * GS;
                const double xr = __shfl(qr, src, SBP_WAVE), xf = __shfl(qf, src, SBP_WAVE);
                const double xu = __shfl(u, src, SBP_WAVE);
                // a zero Hastings sum gives -inf, as in a direct evaluation; the
                // values of vertices that do not move are not used
                lg = log(m == 0 ? xr : m == 1 ? xf : xu);
            }
            const double lnqr = __shfl(lg, 3 * wgrp + 0, SBP_WAVE);
            const double lnqf = __shfl(lg, 3 * wgrp + 1, SBP_WAVE);
            const double lnu = __shfl(lg, 3 * wgrp + 2, SBP_WAVE);
            const double dS = -dL;
            const double lnH = (act && k > 0) ? lnqr - lnqf : 0.0;
            const double z = -a.beta * dS + lnH;
            const bool acc = act && lnu < z;
            const bool tie = act && fabs(z - lnu) < SBP_NEAR_TIE;
            if (gl == 0 && valid) {
                if (!hub) {
                    ++n_prop;
                    if (!act) ++n_self;
                }
                if (acc) {
                    ++n_acc;
                    s_dS += dS;
                }
                n_tie += tie ? 1 : 0;
                if constexpr (ENDS) ((unsigned char *)a.nb)[v] = acc ? (unsigned char)s : 0xffu;
                else ((int *)a.nb)[v] = acc ? s : -1;
                if constexpr (TRACE) if (!hub) {
                    const int uu = a.voff + v;
                    if (tr.prop) tr.prop[uu] = act ? s : r;
                    if (tr.dS) tr.dS[uu] = act ? dS : 0.0;
                    if (tr.lnH) tr.lnH[uu] = act ? lnH : 0.0;
                    if (tr.margin) tr.margin[uu] = act ? z - lnu : 0.0;
                    if (tr.accept) tr.accept[uu] = acc ? 1 : 0;
                    // -1 no-op, else accepted (bit 0) and near tie (bit 1)
                    if (tr.status) tr.status[uu] = act ? (acc ? 1 : 0) + (tie ? 2 : 0) : -1;
                }
            }
        }
    }
    if (!a.stats_part) return;  // uniform: the multi-graph pass keeps no statistics
    n_prop = wave_sum_i64(n_prop);
    n_self = wave_sum_i64(n_self);
    n_acc = wave_sum_i64(n_acc);
    n_tie = wave_sum_i32(n_tie);
    s_dS = wave_sum(s_dS);
    __syncthreads();
    if (lane == 0) {
        L.wst[4 * wv + 0] = n_prop;
        L.wst[4 * wv + 1] = n_self;
        L.wst[4 * wv + 2] = n_acc;
        L.wst[4 * wv + 3] = n_tie;
        L.wsd[wv] = s_dS;
    }
    __syncthreads();
    if (tid == 0) {
        long long p = 0, sp = 0, ac = 0, ti = 0;
        double sd = 0.0;
        for (int w = 0; w < EVAL_T / 64; ++w) {
            p += L.wst[4 * w + 0];
            sp += L.wst[4 * w + 1];
            ac += L.wst[4 * w + 2];
            ti += L.wst[4 * w + 3];
            sd += L.wsd[w];
        }
        a.stats_part[4 * blockIdx.x + 0] = p;
        a.stats_part[4 * blockIdx.x + 1] = sp;
        a.stats_part[4 * blockIdx.x + 2] = ac;
        a.stats_part[4 * blockIdx.x + 3] = ti;
        a.sum_part[blockIdx.x] = sd;
    }
}

template <bool ENDS, bool TRACE, int CM>
__global__ void __launch_bounds__(EVAL_T) __attribute__((amdgpu_waves_per_eu(EvalLds<CM>::WAVES))) k_dense_eval(EvalArgs a, SweepTraceDev tr) {
    __shared__ EvalLds<CM> L;
    eval_body<ENDS, TRACE, CM>(L, a, tr, StridedChunks{(int)blockIdx.x, (int)gridDim.x, 0});
}

// Many graphs in one persistent launch, each with its own work queue of chunk
// runs (ctr[g] counts the runs taken, nruns[g] of them exist).  A workgroup
// starts at the graph its index falls in (spread by work), drains that
// graph's queue, then moves on to the next graph with work left; it ends after
// finding every queue empty once in a row, so every workgroup exits.  The
// graph's blockmodel is staged in LDS each time a workgroup starts on a
// graph.  Decisions are ints (the labels are gathered, no end bytes), no
// statistics and no trace.
template <int CM>
__global__ void __launch_bounds__(EVAL_T) __attribute__((amdgpu_waves_per_eu(EvalLds<CM>::WAVES))) k_dense_eval_multi(const EvalArgs *__restrict__ A,
                                                               const int *__restrict__ nruns,
                                                               const int *__restrict__ gstart, int *__restrict__ ctr,
                                                               int D, int run_len) {
    __shared__ EvalLds<CM> L;
    __shared__ int pull;
    // first graph: the one whose share of the grid holds this workgroup
    int g = 0;
    {
        int lo = 0, hi = D - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (gstart[mid] <= (int)blockIdx.x) lo = mid; else hi = mid - 1;
        }
        g = lo;
    }
    int misses = 0;
    while (misses < D) {
        if (threadIdx.x == 0) pull = atomicAdd(&ctr[g], 1);
        __syncthreads();
        const int run = __builtin_amdgcn_readfirstlane(pull);
        if (run < nruns[g]) {
            misses = 0;
            const EvalArgs a = A[g];
            eval_body<false, false, CM>(L, a, SweepTraceDev{},
                                        QueueChunks{&ctr[g], &pull, run_len, run * run_len, 0, 0});
        } else {
            ++misses;
        }
        __syncthreads();  // the LDS and the pulled index are free again
        g = g + 1 == D ? 0 : g + 1;
    }
}

// Dense copy of one graph's part of the union sparse blockmodel (one
// workgroup per graph): M from its C rows, f(M), block degrees; also empties
// the graph's work queue for the evaluation that follows.
struct ToDense {
    int boff, C;
    int *M;
    double *fM;
    int *dout, *din;
};
__global__ void __launch_bounds__(256) k_to_dense(const ToDense *__restrict__ J, SparseBM bm,
                                                  const double *__restrict__ tab, unsigned fmax,
                                                  int *__restrict__ ctr) {
    const ToDense j = J[blockIdx.x];
    const int C = j.C, CC = C * C, tid = threadIdx.x;
    for (int i = tid; i < CC; i += 256) j.M[i] = 0;
    __syncthreads();
    for (int a = 0; a < C; ++a) {
        const int p0 = bm.rptr[j.boff + a], p1 = bm.rptr[j.boff + a + 1];
        for (int q = p0 + tid; q < p1; q += 256) j.M[a * C + (bm.rcol[q] - j.boff)] = bm.rval[q];
    }
    __syncthreads();
    for (int i = tid; i < CC; i += 256) j.fM[i] = fx(tab, fmax, j.M[i]);
    if (tid < C) {
        j.dout[tid] = bm.dout[j.boff + tid];
        j.din[tid] = bm.din[j.boff + tid];
    }
    if (tid == 0) ctr[blockIdx.x] = 0;
}

// After the decisions of a single-batch sweep: every edge end once, chunks of
// CHU consecutive vertices per workgroup (a workgroup per CU, each with a
// balanced range of vertices, so mostly one chunk each).  An out-edge (v, u) moves one count of
// M from (old v, old u) to (new v, new u) when either endpoint moved (LDS
// delta, flushed with integer atomics); every end byte takes the far end's new
// block; the labels of the chunk's vertices take their decisions.  The
// decisions are read from nb (never from the labels being rewritten), so the
// workgroups need no ordering.  A thread takes 8 consecutive ends of the
// chunk (its out-ends, then its in-ends) and issues all their loads and
// decision gathers before any use.
constexpr int CHU = 1024;    // vertices per chunk of the update
constexpr int UPD_T = 1024;  // threads per update workgroup, one workgroup per CU
constexpr int UPD_GRID_V = 512;  // at least this many vertices per workgroup (and at most one per CU)
static_assert(CHU <= UPD_T, "a chunk's vertices are loaded by one thread each");
// A thread takes an 8-aligned block of 8 consecutive end positions of the
// chunk (its out-ends, then its in-ends): with VEC (16-byte aligned id
// arrays) the ids come in two 16-byte loads, the end bytes in one 8-byte load
// (the byte arrays are padded to 256).  Bytes outside the chunk are read but
// neither used nor written: their owners are other workgroups.  The decisions
// of vertices [0, sl) are copied into LDS first (sl fills what the LDS of the
// CU has left), so the far-end lookups of those vertices are LDS reads; the
// rest are gathered.
template <bool VEC>
__global__ void __launch_bounds__(UPD_T) k_dense_update(GDev g, DenseBM bm, const unsigned char *__restrict__ nb,
                                                        int *__restrict__ delta, int sl,
                                                        const long long *__restrict__ stats_part, int nstats,
                                                        int moved_share) {
    const int *ub = bm.bounds;
    const bool ranged = ub[0] == (int)gridDim.x;
    const int rb0 = ranged ? ub[1 + blockIdx.x] : 0, rb1 = ranged ? ub[2 + blockIdx.x] : 0;
    extern __shared__ __align__(16) char smem[];
    const int C = g.C, CC = C * C, tid = threadIdx.x;
    int *dl = (int *)smem;
    int *op = dl + CC;       // [CHU + 1] first out-end; op[nv] = end of the chunk's out-ends
    int *ip = op + CHU + 1;  // [CHU + 1] first in-end
    int *a0 = ip + CHU + 1;  // [CHU] old label
    int *a1 = a0 + CHU;      // [CHU] new label
    int &s_moved = a1[CHU];  // the workgroup's choice of update
    unsigned char *nbs = (unsigned char *)smem + ((sizeof(int) * (CC + 4 * CHU + 3) + 15) & ~(size_t)15);
    unsigned char *__restrict__ nlo = bm.nl;
    unsigned char *__restrict__ nli = bm.nl + bm.nl_in;
    // Few moves (at most moved_share / 1024 of the vertices, counted from the
    // evaluation's partials) and verified mirrors: only the moved vertices'
    // edges change M, so each workgroup finds the moved vertices of its share
    // and adds their edges' changes (an edge counted by its source when the
    // source moved, else by its target), reading old blocks from the end
    // bytes, which this kernel then leaves untouched; the final kernel writes
    // the new blocks into the mirrors.
    {
        long long acc = 0;
        for (int w = tid; w < nstats; w += UPD_T) acc += stats_part[4 * w + 2];
        acc = wave_sum_i64(acc);
        long long *red = (long long *)smem;  // the histogram's space, cleared below
        if ((tid & 63) == 0) red[tid >> 6] = acc;
        __syncthreads();
        if (tid == 0) {
            long long t = 0;
            for (int w = 0; w < UPD_T / 64; ++w) t += red[w];
            s_moved = bm.flags[0] == 1 && moved_share >= 0 && t * 1024 <= (long long)moved_share * g.n;
        }
        __syncthreads();
    }
    if (blockIdx.x == 0 && tid == 0) bm.flags[1] = s_moved;
    if (s_moved) {
        for (int i = tid; i < CC; i += UPD_T) dl[i] = 0;
        __syncthreads();
        const int lane = tid & 63, wv = tid >> 6;
        const int v0 = (int)((long long)g.n * blockIdx.x / gridDim.x);
        const int v1 = (int)((long long)g.n * (blockIdx.x + 1) / gridDim.x);
        const int elast = max(g.e - 1, 0);
        for (int tb = v0 + wv * 64; tb < v1; tb += UPD_T) {
            const int v = tb + lane;
            const unsigned x = v < v1 ? nb[v] : 0xffu;
            // every moved lane's label and end ranges in one round trip
            const int vc = min(v, g.n - 1);
            const int la = g.lab[vc], lo0 = g.out_ptr[vc], lo1 = g.out_ptr[vc + 1];
            const int li0 = g.in_ptr[vc], li1 = g.in_ptr[vc + 1];
            for (uint64_t todo = __ballot(x != 0xffu); todo; todo &= todo - 1) {
                const int l = __builtin_ctzll(todo);
                const int vv = tb + l;
                const int xn = __shfl((int)x, l, 64);
                const int a = __shfl(la, l, 64);
                const int o0 = __shfl(lo0, l, 64), ko = __shfl(lo1, l, 64) - o0;
                const int i0 = __shfl(li0, l, 64), ki = __shfl(li1, l, 64) - i0;
                // out-end j and in-end j together; loads unconditional (positions
                // clamped into the arrays), so both ends' reads overlap
                for (int j = lane; j < max(ko, ki); j += 64) {
                    const bool ho = j < ko, hi = j < ki;
                    const int p = min(o0 + j, elast), q = min(i0 + j, elast);
                    const unsigned bo = nlo[p], bi = nli[q];
                    const unsigned xu = nb[g.out_idx[p]], xw = nb[g.in_idx[q]];
                    if (ho) {
                        if (bo == 0xffu) {  // self-loop: (a, a) -> (x, x)
                            atomicAdd(&dl[a * C + a], -1);
                            atomicAdd(&dl[xn * C + xn], 1);
                        } else {
                            const int bn = xu != 0xffu ? (int)xu : (int)bo;
                            atomicAdd(&dl[a * C + (int)bo], -1);
                            atomicAdd(&dl[xn * C + bn], 1);
                        }
                    }
                    if (hi && bi != 0xffu && xw == 0xffu) {  // else counted at the (moved) source
                        atomicAdd(&dl[(int)bi * C + a], -1);
                        atomicAdd(&dl[(int)bi * C + xn], 1);
                    }
                }
                if (lane == 0) g.lab[vv] = xn;
            }
        }
        __syncthreads();
        for (int i = tid; i < CC; i += UPD_T)
            if (dl[i]) atomicAdd(&delta[i], dl[i]);
        return;
    }
    for (int i = tid; i < CC; i += UPD_T) dl[i] = 0;
    const int nchunks = (g.n + CHU - 1) / CHU;
    for (int ci = 0;; ++ci) {
        int base, nv;
        if (ranged) {  // the workgroup's own range of vertices, in chunks
            base = rb0 + ci * CHU;
            if (base >= rb1) break;
            nv = min(CHU, rb1 - base);
        } else {
            const int chunk = blockIdx.x + ci * gridDim.x;
            if (chunk >= nchunks) break;
            base = chunk * CHU;
            nv = min(CHU, g.n - base);
        }
        __syncthreads();
        // the chunk's head loads go out before the first chunk's copy of the
        // staged decisions, so the two overlap
        const bool hv = tid < nv;
        const int vh = base + (hv ? tid : 0);
        const int h_op = g.out_ptr[vh], h_ip = g.in_ptr[vh], h_old = g.lab[vh];
        const unsigned h_x = nb[vh];
        const int h_op1 = tid == nv - 1 ? g.out_ptr[vh + 1] : 0, h_ip1 = tid == nv - 1 ? g.in_ptr[vh + 1] : 0;
        if (ci == 0)
            for (int i = tid; i < sl / 16; i += UPD_T) ((uint4 *)nbs)[i] = ((const uint4 *)nb)[i];
        if (hv) {
            op[tid] = h_op;
            ip[tid] = h_ip;
            if (tid == nv - 1) {  // the ends of the chunk's ranges
                op[nv] = h_op1;
                ip[nv] = h_ip1;
            }
            a0[tid] = h_old;
            a1[tid] = h_x != 0xffu ? (int)h_x : h_old;
            if (h_x != 0xffu) g.lab[vh] = (int)h_x;
        }
        __syncthreads();
        const int o0 = op[0], o1 = op[nv], i0 = ip[0], i1 = ip[nv];
        const int bo0 = o0 >> 3, nbo = o1 > o0 ? ((o1 + 7) >> 3) - bo0 : 0;
        const int bi0 = i0 >> 3, nbi = i1 > i0 ? ((i1 + 7) >> 3) - bi0 : 0;
        const int nbt = nbo + nbi;
        // Block rr of the chunk: its first position, run and owner array.
        // Ids, end bytes and the far ends' decisions of a thread's two blocks
        // are all loaded before either block is counted.
        struct Blk {
            bool out;
            int p0, lo, hi;
            unsigned b[8], x[8];
        };
        auto load_blk = [&](int rr, bool mine, Blk &k) {
            k.out = rr < nbo;
            k.p0 = (k.out ? bo0 + rr : bi0 + (rr - nbo)) * 8;
            k.lo = k.out ? o0 : i0;
            k.hi = k.out ? o1 : i1;
            const int *__restrict__ idx = k.out ? g.out_idx : g.in_idx;
            const unsigned char *__restrict__ nlp = k.out ? nlo : nli;
            int u[8];
            if (VEC && k.p0 + 8 <= g.e) {
                const int4 A = *(const int4 *)(idx + k.p0), B = *(const int4 *)(idx + k.p0 + 4);
                u[0] = A.x; u[1] = A.y; u[2] = A.z; u[3] = A.w;
                u[4] = B.x; u[5] = B.y; u[6] = B.z; u[7] = B.w;
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) u[q] = (k.p0 + q >= k.lo && k.p0 + q < k.hi) ? idx[k.p0 + q] : 0;
            }
            const uint2 bw = *(const uint2 *)(nlp + k.p0);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const bool in_run = mine && k.p0 + q >= k.lo && k.p0 + q < k.hi;
                k.b[q] = in_run ? (((q < 4 ? bw.x : bw.y) >> (8 * (q & 3))) & 0xffu) : 0x100u;  // 0x100: not ours
            }
#pragma unroll
            for (int q = 0; q < 8; ++q)
                k.x[q] = k.b[q] < 0xffu ? (u[q] < sl ? (unsigned)nbs[u[q]] : (unsigned)nb[u[q]]) : 0xffu;
        };
        auto count_blk = [&](const Blk &k) {
            unsigned char *__restrict__ nlp = k.out ? nlo : nli;
            int w = 0, nxt = 0;
            if (k.out) {  // owner of the first position of the block in the chunk, then a forward walk
                const int pf = max(k.lo, k.p0);
                int l = 0, h = nv - 1;
                while (l < h) {
                    const int mid = (l + h + 1) >> 1;
                    if (op[mid] <= pf) l = mid; else h = mid - 1;
                }
                w = l;
                nxt = op[l + 1];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (k.b[q] == 0x100u) continue;
                const unsigned bn = k.x[q] != 0xffu ? k.x[q] : k.b[q];
                if (bn != k.b[q]) nlp[k.p0 + q] = (unsigned char)bn;
                if (!k.out) continue;
                while (k.p0 + q >= nxt) nxt = op[++w + 1];
                const int va = a0[w], vb = a1[w];
                const int ua = k.b[q] == 0xffu ? va : (int)k.b[q];  // a self-loop's far end is the vertex
                const int ub = k.b[q] == 0xffu ? vb : (int)bn;
                if (va != vb || ua != ub) {
                    atomicAdd(&dl[va * C + ua], -1);
                    atomicAdd(&dl[vb * C + ub], 1);
                }
            }
        };
        for (int rr = tid; rr < nbt; rr += 2 * UPD_T) {
            const int rr2 = rr + UPD_T;
            const bool two = rr2 < nbt;
            Blk k1, k2;
            load_blk(rr, true, k1);
            load_blk(two ? rr2 : rr, two, k2);  // without a second block: the first again, nothing of it counted
            count_blk(k1);
            if (two) count_blk(k2);
        }
    }
    __syncthreads();
    for (int i = tid; i < CC; i += UPD_T)
        if (dl[i]) atomicAdd(&delta[i], dl[i]);
}

// Change of M from the accepted moves of one batch, exact for moves of
// adjacent vertices: edge (u, w) goes from (old u, old w) to (new u, new w);
// it is counted by its source when the source moved, else by its target.
__global__ void __launch_bounds__(256) k_dense_delta(GDev g, const int *__restrict__ nb, int *__restrict__ delta) {
    __shared__ int dl[DC * DC];
    const int C = g.C, CC = C * C;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int i = tid; i < CC; i += blockDim.x) dl[i] = 0;
    __syncthreads();
    const int nbc = (g.n - g.batch + g.n_batches - 1) / g.n_batches;
    for (int base = (blockIdx.x * 4 + wv) * 64; base < nbc; base += gridDim.x * 4 * 64) {
        const int my_idx = base + lane;
        const int my_v = g.batch + my_idx * g.n_batches;
        const int my_x = my_idx < nbc ? nb[my_v] : -1;
        uint64_t moved = __ballot(my_x >= 0);
        while (moved) {
            const int b = __builtin_ctzll(moved);
            moved &= moved - 1;
            const int v = __shfl(my_v, b, SBP_WAVE), x = __shfl(my_x, b, SBP_WAVE);
            const int r = g.lab[v];
            const int op = g.out_ptr[v], kout = g.out_ptr[v + 1] - op;
            const int ip = g.in_ptr[v], kin = g.in_ptr[v + 1] - ip;
            for (int j = lane; j < kout; j += 64) {
                const int w = g.out_idx[op + j];
                const int bo = g.lab[w];
                const bool wmoved = (w % g.n_batches) == g.batch && nb[w] >= 0;
                const int bn = wmoved ? nb[w] : bo;
                atomicAdd(&dl[r * C + bo], -1);
                atomicAdd(&dl[x * C + bn], 1);
            }
            for (int j = lane; j < kin; j += 64) {
                const int u = g.in_idx[ip + j];
                if ((u % g.n_batches) == g.batch && nb[u] >= 0) continue;
                const int a = g.lab[u];
                atomicAdd(&dl[a * C + r], -1);
                atomicAdd(&dl[a * C + x], 1);
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < CC; i += blockDim.x)
        if (dl[i]) atomicAdd(&delta[i], dl[i]);
}

// Labels of the accepted moves of one batch of several.
__global__ void k_dense_apply(GDev g, const int *__restrict__ nb) {
    const int nbc = (g.n - g.batch + g.n_batches - 1) / g.n_batches;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nbc; i += gridDim.x * blockDim.x) {
        const int v = g.batch + i * g.n_batches;
        const int x = nb[v];
        if (x >= 0) g.lab[v] = x;
    }
}

// Running sum over b' <= lane of e_t,b' = M_t,b' + M_b',t (lane b <-> block b),
// the table a block proposal draws from; every lane of the wave takes part.
__device__ __forceinline__ long long running_e(const int *__restrict__ M, int C, int t, int lane) {
    long long x = lane < C ? (long long)M[t * C + lane] + M[lane * C + t] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long y = __shfl_up(x, o, SBP_WAVE);
        if (lane >= o) x += y;
    }
    return x;
}

// Hub order keys: descending degree (out + in edge ends) in bits 32-46, the
// vertex id below.  The keys are written in id order and sorted stably on the
// degree bits alone, so ties keep ascending ids.
__global__ void k_hub_keys(GDev g, uint64_t *__restrict__ keys, int *__restrict__ hubrank) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += gridDim.x * blockDim.x) {
        const int deg = (g.out_ptr[v + 1] - g.out_ptr[v]) + (g.in_ptr[v + 1] - g.in_ptr[v]);
        keys[v] = ((uint64_t)(SBP_MAX_DEGREE_DEV - deg) << 32) | (uint32_t)v;
        hubrank[v] = 0;
    }
}
// The first nh sorted vertices: order, rank (1-based), out | in << 16 end
// counts and the offsets of their edge ends in the code arrays (an exclusive
// scan of the degrees, one workgroup, nh <= SBP_HUBS_MAX).
constexpr int MARK_T = 1024;
__global__ void __launch_bounds__(MARK_T) k_hub_mark(GDev g, const uint64_t *__restrict__ keys, int nh,
                                                     int *__restrict__ order, int *__restrict__ hubrank,
                                                     int *__restrict__ kk, int *__restrict__ hoff) {
    __shared__ int part[MARK_T];
    constexpr int PER = SBP_HUBS_MAX / MARK_T;
    const int tid = threadIdx.x;
    int deg[PER], sum = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = tid * PER + q;
        deg[q] = 0;
        if (i < nh) {
            const int v = (int)(uint32_t)keys[i];
            const int ko = g.out_ptr[v + 1] - g.out_ptr[v], ki = g.in_ptr[v + 1] - g.in_ptr[v];
            order[i] = v;
            hubrank[v] = i + 1;
            kk[i] = ko | (ki << 16);
            deg[q] = ko + ki;
        }
        sum += deg[q];
    }
    part[tid] = sum;
    __syncthreads();
    for (int o = 1; o < MARK_T; o <<= 1) {  // inclusive scan of the thread sums
        const int x = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += x;
        __syncthreads();
    }
    int run = part[tid] - sum;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = tid * PER + q;
        if (i < nh) hoff[i] = run;
        run += deg[q];
    }
    if (tid == MARK_T - 1) hoff[nh] = part[MARK_T - 1];
}
// Neighbour codes of every hub edge end, contiguous per hub (a workgroup per
// hub): the far end's block (>= 0) for a vertex that is no hub (its label
// does not change during the pass), -rank for a hub, HUB_SELF for a self-loop;
// mpos holds the position of the mirror end byte (in-ends for out-ends and
// the reverse).
constexpr int HUB_SELF = -(1 << 20);
__global__ void __launch_bounds__(256) k_hub_codes(GDev g, DenseBM bm, const int *__restrict__ order,
                                                   const int *__restrict__ kk, const int *__restrict__ hoff,
                                                   const int *__restrict__ hubrank, int *__restrict__ codes,
                                                   int *__restrict__ mpos) {
    const int i = blockIdx.x, v = order[i], kout = kk[i] & 0xffff, k = kout + (kk[i] >> 16), h0 = hoff[i];
    const int op = g.out_ptr[v], ip = g.in_ptr[v];
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        const bool out = j < kout;
        const int p = out ? op + j : ip + (j - kout);
        const int u = out ? g.out_idx[p] : g.in_idx[p];
        const int hr = hubrank[u];
        codes[h0 + j] = u == v ? HUB_SELF : hr > 0 ? -hr : g.lab[u];
        mpos[h0 + j] = out ? bm.mir_o[p] : bm.mir_i[p];
    }
}

// End bytes from the labels, only when the mirrors could not be verified (the
// sequential pass then leaves the bytes pointing at moved hubs stale).
__global__ void __launch_bounds__(256) k_dense_ends_unmirrored(GDev g, DenseBM bm) {
    if (bm.flags[0] == 1) return;
    const int lane = threadIdx.x & 63;
    unsigned char *nlo = bm.nl, *nli = bm.nl + bm.nl_in;
    for (int v = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; v < g.n; v += (gridDim.x * blockDim.x) >> 6) {
        const int o1 = g.out_ptr[v + 1], i1 = g.in_ptr[v + 1];
        for (int j = g.out_ptr[v] + lane; j < o1; j += 64) {
            const int u = g.out_idx[j];
            nlo[j] = u == v ? 0xffu : (unsigned char)g.lab[u];
        }
        for (int j = g.in_ptr[v] + lane; j < i1; j += 64) {
            const int u = g.in_idx[j];
            nli[j] = u == v ? 0xffu : (unsigned char)g.lab[u];
        }
    }
}

// Hybrid sweep, sequential part (Sec. II-B): the hubs order[0..nh) move one at
// a time in that order, each evaluated against the state the previous ones
// left and applied at once.  One workgroup keeps M, the block degrees and the
// hubs' labels in LDS.  A hub's neighbour blocks come from its precomputed
// codes (a hub neighbour's block from LDS: it may have moved in this pass),
// loaded one hub ahead so that the loads of the next hub overlap the scoring
// of this one.  The proposal and the scoring are those of the evaluation
// kernel (one lane per block; the corner, degree and Hastings terms of r and
// s on lanes 0-11).  An accepted move updates M, the degrees and the label,
// and writes the new block into the mirrors of the hub's edge ends.  At the
// end M, f(M) and the degrees go back to global memory and the pass's totals
// to statistics slot `slot`.
constexpr int HUBS_T = 256;  // one wave per SIMD
constexpr int HUB_PF = 4;    // ends per thread held one hub ahead (hub degree up to 1024)
struct HubEnds {
    int c[HUB_PF], m[HUB_PF];
};
__device__ __forceinline__ void hub_fetch(const int *__restrict__ codes, const int *__restrict__ mpos, int h0,
                                          int k, int tid, HubEnds &e) {
#pragma unroll
    for (int q = 0; q < HUB_PF; ++q) {
        const int j = tid + q * HUBS_T;
        e.c[q] = j < k ? codes[h0 + j] : 0;
        e.m[q] = j < k ? mpos[h0 + j] : -1;
    }
}
__global__ void __launch_bounds__(HUBS_T) k_dense_hubs(GDev g, DenseBM bm, const int *__restrict__ order, int nh,
                                                       const int *__restrict__ kk, const int *__restrict__ hoff,
                                                       const int *__restrict__ codes, const int *__restrict__ mpos,
                                                       long long *__restrict__ stats_part,
                                                       double *__restrict__ sum_part, int slot, SweepTraceDev tr) {
    __shared__ int Ms[DC * DC];
    __shared__ int dos[DC], dis[DC];
    __shared__ unsigned H[DC];  // out | in << 16 ends of the hub into each block
    __shared__ int hl[SBP_HUBS_MAX];
    __shared__ int s_ell, s_t0, s_dec;
    __shared__ uint64_t s_W[2][3];  // a hub's draw words 1-3 and first index, double-buffered by hub parity
    __shared__ int s_j0[2];
    const int C = g.C, CC = C * C, tid = threadIdx.x, lane = tid & 63;
    const double *tab = bm.ftab;
    const unsigned fmax = bm.ftab_max;
    const double eps = (double)g.eps, epsC = (double)g.eps * (double)C;
    const long long eC = (long long)g.eps * C;
    unsigned char *nlo = bm.nl, *nli = bm.nl + bm.nl_in;
    const bool mirrored = bm.flags[0] == 1;
    // wave 1 draws hub i's words while wave 0 scores hub i - 1
    auto draw_hub = [&](int vv, int kvv, int slot_) {
        const Words4 W = draw_words(g.seed, (uint32_t)vv, sweep_of(g), 0u, 0u);
        const int kk_ = (kvv & 0xffff) + (kvv >> 16);
        if (lane == 0) {
            s_W[slot_][0] = W.w[1];
            s_W[slot_][1] = W.w[2];
            s_W[slot_][2] = W.w[3];
            s_j0[slot_] = kk_ > 0 ? (int)draw_idx(W.w[0], (uint64_t)kk_) : -1;
        }
    };
    for (int i = tid; i < CC; i += HUBS_T) Ms[i] = bm.M[i];
    if (tid < C) {
        dos[tid] = bm.dout[tid];
        dis[tid] = bm.din[tid];
    }
    for (int i = tid; i < nh; i += HUBS_T) hl[i] = g.lab[order[i]];
    long long n_prop = 0, n_self = 0, n_acc = 0, n_tie = 0;
    double s_dS = 0.0;
    // hub i's meta and ends; hub i + 1's meta
    int v = order[0], kv = kk[0], h0 = hoff[0];
    HubEnds E;
    hub_fetch(codes, mpos, h0, (kv & 0xffff) + (kv >> 16), tid, E);
    // complete the first hub's loads here: a first use inside the loop would
    // place the wait there, where it would also drain each next hub's loads
#pragma unroll
    for (int q = 0; q < HUB_PF; ++q) asm volatile("" ::"v"(E.c[q]), "v"(E.m[q]));
    int v_n = nh > 1 ? order[1] : 0, kv_n = nh > 1 ? kk[1] : 0, h0_n = nh > 1 ? hoff[1] : 0;
    if (tid >= 64 && tid < 128) draw_hub(v, kv, 0);
    __syncthreads();
    for (int i = 0; i < nh; ++i) {
        const int r = hl[i];
        const int kout = kv & 0xffff, kin = kv >> 16, k = kout + kin;
        // the next hub's ends and the meta of the one after, in flight during this hub
        HubEnds En;
        hub_fetch(codes, mpos, h0_n, i + 1 < nh ? (kv_n & 0xffff) + (kv_n >> 16) : 0, tid, En);
        const int v_nn = i + 2 < nh ? order[i + 2] : 0, kv_nn = i + 2 < nh ? kk[i + 2] : 0;
        const int h0_nn = i + 2 < nh ? hoff[i + 2] : 0;
        const int j0 = s_j0[i & 1];
        if (tid < C) H[tid] = 0;
        if (tid == 0) {
            s_ell = 0;
            s_t0 = r;
        }
        __syncthreads();
        // neighbour blocks: a self-loop end counts in ell (its block is r)
#pragma unroll
        for (int q = 0; q < HUB_PF; ++q) {
            const int j = tid + q * HUBS_T;
            if (j < k) {
                const int c = E.c[q];
                const bool out = j < kout;
                int b = r;
                if (c == HUB_SELF) {
                    if (out) atomicAdd(&s_ell, 1);
                } else {
                    b = c >= 0 ? c : hl[-c - 1];
                    atomicAdd(&H[b], out ? 1u : 65536u);
                }
                if (j == j0) s_t0 = b;
            }
        }
        for (int j = tid + HUB_PF * HUBS_T; j < k; j += HUBS_T) {  // beyond the prefetched ends
            const int c = codes[h0 + j];
            const bool out = j < kout;
            int b = r;
            if (c == HUB_SELF) {
                if (out) atomicAdd(&s_ell, 1);
            } else {
                b = c >= 0 ? c : hl[-c - 1];
                atomicAdd(&H[b], out ? 1u : 65536u);
            }
            if (j == j0) s_t0 = b;
        }
        __syncthreads();
        if (tid >= 64 && tid < 128 && i + 1 < nh) draw_hub(v_n, kv_n, (i + 1) & 1);
        if (tid < 64) {
            const int t = lane;
            Words4 W;
            W.w[1] = s_W[i & 1][0];
            W.w[2] = s_W[i & 1][1];
            W.w[3] = s_W[i & 1][2];
            int s;
            if (k == 0) {
                s = (int)draw_idx(W.w[2], (uint64_t)C);
            } else {
                const int t0 = s_t0;
                const long long dt = (long long)dos[t0] + dis[t0];
                if (draw_idx(W.w[1], (uint64_t)(dt + eC)) < (uint64_t)eC) {
                    s = (int)draw_idx(W.w[2], (uint64_t)C);
                } else {
                    // the first block whose running sum of e_t0,b = M_t0,b + M_b,t0 exceeds x
                    const int x = (int)draw_idx(W.w[2], (uint64_t)dt);  // dt <= 2e < 2^31
                    int e = t < C ? Ms[t0 * C + t] + Ms[t * C + t0] : 0;
#pragma unroll
                    for (int o = 1; o < 64; o <<= 1) {
                        const int y = __shfl_up(e, o, 64);
                        if (lane >= o) e += y;
                    }
                    const uint64_t hit = __ballot(t < C && e > x);
                    s = hit ? __builtin_ctzll(hit) : r;
                }
            }
            const double lnu = log(draw_unit(W.w[3]));
            const bool act = s != r;
            double dS = 0.0, lnH = 0.0, z = 0.0;
            bool acc = false;
            if (act) {
                // every lane issues its ten f lookups at once (one round trip):
                // its block t's four changed entries before and after, and for
                // lanes 0-7 one corner entry or block degree; an unused slot
                // looks up f(0) - f(0), an exact zero
                double dL = 0.0, qf = 0.0, qr = 0.0;
                const bool bt = t < C && t != r && t != s;
                const int tc = bt ? t : 0;
                const unsigned hv = bt ? H[tc] : 0u;
                const int ko = (int)(hv & 0xffffu), ki = (int)(hv >> 16);
                const int Mrt = Ms[r * C + tc], Mst = Ms[s * C + tc], Mtr = Ms[tc * C + r], Mts = Ms[tc * C + s];
                const unsigned hr = H[r], hs = H[s];
                const int ko_r = (int)(hr & 0xffffu), ki_r = (int)(hr >> 16);
                const int ko_s = (int)(hs & 0xffffu), ki_s = (int)(hs >> 16);
                const int ell = s_ell;
                const int Mrr = Ms[r * C + r], Mrs = Ms[r * C + s], Msr = Ms[s * C + r], Mss = Ms[s * C + s];
                const int drr = -ko_r - ki_r - ell, drs = -ko_s + ki_r, dsr = ko_r - ki_s, dss = ko_s + ki_s + ell;
                const int dor = dos[r], dos_ = dos[s], dir = dis[r], dis_ = dis[s];
                int cx = 0, cy = 0;
                switch (lane) {
                    case 0: cx = Mrr + drr, cy = Mrr; break;
                    case 1: cx = Mrs + drs, cy = Mrs; break;
                    case 2: cx = Msr + dsr, cy = Msr; break;
                    case 3: cx = Mss + dss, cy = Mss; break;
                    case 4: cx = dor - kout, cy = dor; break;
                    case 5: cx = dos_ + kout, cy = dos_; break;
                    case 6: cx = dir - kin, cy = dir; break;
                    case 7: cx = dis_ + kin, cy = dis_; break;
                    default: break;
                }
                const double f0 = fx(tab, fmax, ko ? Mrt - ko : 0), g0 = fx(tab, fmax, ko ? Mrt : 0);
                const double f1 = fx(tab, fmax, ko ? Mst + ko : 0), g1 = fx(tab, fmax, ko ? Mst : 0);
                const double f2 = fx(tab, fmax, ki ? Mtr - ki : 0), g2 = fx(tab, fmax, ki ? Mtr : 0);
                const double f3 = fx(tab, fmax, ki ? Mts + ki : 0), g3 = fx(tab, fmax, ki ? Mts : 0);
                const double fc = fx(tab, fmax, cx), gc = fx(tab, fmax, cy);
                // Hastings terms while the lookups are in flight
                if (ko | ki) {
                    const double kt = (double)(ko + ki), den = (double)(dos[tc] + dis[tc]) + epsC;
                    qf += kt * (((double)(Mts + Mst) + eps) / den);
                    qr += kt * (((double)(Mtr - ki + Mrt - ko) + eps) / den);
                }
                if (lane >= 8 && lane < 12) {  // t = r and t = s
                    const double kd = (double)k;
                    const double d_r = (double)dor + (double)dir, d_s = (double)dos_ + (double)dis_;
                    int w, num;
                    double den;
                    switch (lane) {
                        case 8: w = ko_r + ki_r + 2 * ell, num = Mrs + Msr, den = d_r + epsC; break;
                        case 9: w = ko_s + ki_s, num = 2 * Mss, den = d_s + epsC; break;
                        case 10: w = ko_r + ki_r, num = 2 * (Mrr + drr), den = d_r - kd + epsC; break;
                        default: w = ko_s + ki_s + 2 * ell, num = Msr + dsr + Mrs + drs, den = d_s + kd + epsC; break;
                    }
                    if (w) {
                        const double q = (double)w * (((double)num + eps) / den);
                        if (lane < 10) qf += q; else qr += q;
                    }
                }
                dL = ((f0 - g0) + (f1 - g1)) + ((f2 - g2) + (f3 - g3)) + (lane < 4 ? fc - gc : gc - fc);
                dL = grp_sum<32>(dL);
                qf = grp_sum<32>(qf);
                qr = grp_sum<32>(qr);
                dL += __shfl_xor(dL, 32, 64);
                qf += __shfl_xor(qf, 32, 64);
                qr += __shfl_xor(qr, 32, 64);
                dS = -dL;
                lnH = k > 0 ? log(qr) - log(qf) : 0.0;
                z = -g.beta * dS + lnH;
                acc = lnu < z;
            }
            if (lane == 0) {
                const bool tie = act && fabs(z - lnu) < SBP_NEAR_TIE;
                ++n_prop;
                if (!act) ++n_self;
                if (acc) {
                    ++n_acc;
                    s_dS += dS;
                }
                n_tie += tie ? 1 : 0;
                const int uu = g.voff + v;
                if (tr.prop) tr.prop[uu] = s;
                if (tr.dS) tr.dS[uu] = dS;
                if (tr.lnH) tr.lnH[uu] = lnH;
                if (tr.margin) tr.margin[uu] = act ? z - lnu : 0.0;
                if (tr.accept) tr.accept[uu] = acc ? 1 : 0;
                if (tr.status) tr.status[uu] = act ? (acc ? 1 : 0) + (tie ? 2 : 0) : -1;
                s_dec = acc ? s : -1;
            }
        }
        __syncthreads();
        const int sd = s_dec;
        if (sd >= 0) {  // apply at once
            if (tid < C) {
                const unsigned hv = H[tid];
                const int ko = (int)(hv & 0xffffu), ki = (int)(hv >> 16);
                if (ko) {
                    atomicAdd(&Ms[r * C + tid], -ko);
                    atomicAdd(&Ms[sd * C + tid], ko);
                }
                if (ki) {
                    atomicAdd(&Ms[tid * C + r], -ki);
                    atomicAdd(&Ms[tid * C + sd], ki);
                }
            }
            if (tid == 0) {
                const int ell = s_ell;
                if (ell) {
                    atomicAdd(&Ms[r * C + r], -ell);
                    atomicAdd(&Ms[sd * C + sd], ell);
                }
                dos[r] -= kout;
                dos[sd] += kout;
                dis[r] -= kin;
                dis[sd] += kin;
                hl[i] = sd;
                g.lab[v] = sd;
            }
            if (mirrored) {  // the end bytes that point at v: in-end bytes of out-ends, and the reverse
#pragma unroll
                for (int q = 0; q < HUB_PF; ++q) {
                    const int j = tid + q * HUBS_T;
                    const int m = E.m[q];
                    if (j < k && E.c[q] != HUB_SELF && (unsigned)m < (unsigned)g.e)
                        (j < kout ? nli : nlo)[m] = (unsigned char)sd;
                }
                for (int j = tid + HUB_PF * HUBS_T; j < k; j += HUBS_T) {
                    const int m = mpos[h0 + j];
                    if (codes[h0 + j] != HUB_SELF && (unsigned)m < (unsigned)g.e)
                        (j < kout ? nli : nlo)[m] = (unsigned char)sd;
                }
            }
        }
        __syncthreads();
        E = En;
        v = v_n;
        kv = kv_n;
        h0 = h0_n;
        v_n = v_nn;
        kv_n = kv_nn;
        h0_n = h0_nn;
    }
    for (int i = tid; i < CC; i += HUBS_T) {
        bm.M[i] = Ms[i];
        bm.fM[i] = fx(tab, fmax, Ms[i]);
    }
    if (tid < C) {
        bm.dout[tid] = dos[tid];
        bm.din[tid] = dis[tid];
    }
    if (tid == 0) {
        stats_part[4 * slot + 0] = n_prop;
        stats_part[4 * slot + 1] = n_self;
        stats_part[4 * slot + 2] = n_acc;
        stats_part[4 * slot + 3] = n_tie;
        sum_part[slot] = s_dS;
    }
}

// Merge scoring on the dense tier, wave per block c, lane t <-> block t.
__global__ void __launch_bounds__(256) k_dense_merge(GDev g, DenseBM bm, int *__restrict__ partner,
                                                    double *__restrict__ dS, double *__restrict__ dSl) {
    const int C = g.C, lane = threadIdx.x & 63;
    const int c = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (c >= C) return;
    const long long eC = (long long)g.eps * C;
    const long long dc = (long long)bm.dout[c] + bm.din[c];
    int best = -1;
    double bestL = 0.0;
    long long bestkey = INT64_MAX;
    for (int j = 0; j < g.proposals && C > 1; ++j) {
        const Words4 W = draw_words(g.seed, (uint32_t)c, g.phase, (uint32_t)(2 * j), 1u);
        int cp;
        if (dc == 0) {
            const int kk = (int)draw_idx(W.w[2], (uint64_t)(C - 1));
            cp = kk + (kk >= c);
        } else {
            const long long x0 = draw_idx(W.w[0], (uint64_t)dc);
            const int t = __builtin_ctzll(__ballot(lane < C && running_e(bm.M, C, c, lane) > x0));
            const long long dt = (long long)bm.dout[t] + bm.din[t];
            if (draw_idx(W.w[1], (uint64_t)(dt + eC)) < eC) {
                const int kk = (int)draw_idx(W.w[2], (uint64_t)(C - 1));
                cp = kk + (kk >= c);
            } else {
                const long long x2 = draw_idx(W.w[2], (uint64_t)dt);
                cp = __builtin_ctzll(__ballot(lane < C && running_e(bm.M, C, t, lane) > x2));
            }
        }
        if (cp == c) continue;
        double acc = 0.0;
        const int t = lane;
        if (t < C && t != c && t != cp) {
            const int x = bm.M[c * C + t], y = bm.M[cp * C + t];
            if (x && y) acc += xlogx((double)(x + y)) - xlogx((double)x) - xlogx((double)y);
            const int xc = bm.M[t * C + c], yc = bm.M[t * C + cp];
            if (xc && yc) acc += xlogx((double)(xc + yc)) - xlogx((double)xc) - xlogx((double)yc);
        }
        if (lane == 0) {
            const int a = bm.M[c * C + c], b = bm.M[c * C + cp], e = bm.M[cp * C + c], f = bm.M[cp * C + cp];
            acc += xlogx((double)(a + b + e + f)) - xlogx((double)a) - xlogx((double)b) - xlogx((double)e) -
                   xlogx((double)f);
            const double oa = bm.dout[c], ob = bm.dout[cp], ia = bm.din[c], ib = bm.din[cp];
            acc -= xlogx(oa + ob) - xlogx(oa) - xlogx(ob);
            acc -= xlogx(ia + ib) - xlogx(ia) - xlogx(ib);
        }
        const double local = -wave_sum(acc);
        const long long key = merge_rank(local);
        if (key < bestkey) {
            bestkey = key;
            best = cp;
            bestL = local;
        }
    }
    if (lane == 0) {
        const double inf = __builtin_huge_val();
        partner[c] = best;
        if (dSl) dSl[c] = best < 0 ? inf : bestL;
        const double off = C > 1 ? model_terms_d((double)g.e, (double)g.n, (double)(C - 1)) -
                                       model_terms_d((double)g.e, (double)g.n, (double)C)
                                 : 0.0;
        dS[c] = best < 0 ? inf : bestL + off;
    }
}

int g_dense_wgs = 0;

}  // namespace

// LDS one workgroup may use (the device's limit, queried once; opting the
// update kernel in to more than 64 KB of dynamic LDS).
int g_lds_block = 0;
int dense_lds_per_block() {
    if (g_lds_block == 0) {
        int dev = 0, v = 65536;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0) {
            if (v > LDS_CU) v = LDS_CU;
        } else {
            v = 65536;
        }
        // the update's dynamic LDS may take all the CU has (it keeps no static
        // LDS); where the runtime refuses that, the default limit holds
        if (hipFuncSetAttribute((const void *)k_dense_update<true>, hipFuncAttributeMaxDynamicSharedMemorySize, v) !=
                hipSuccess ||
            hipFuncSetAttribute((const void *)k_dense_update<false>, hipFuncAttributeMaxDynamicSharedMemorySize, v) !=
                hipSuccess) {
            (void)hipGetLastError();
            v = 65536;
        }
        g_lds_block = v;
    }
    return g_lds_block;
}

int dense_workgroups() {
    if (g_dense_wgs == 0) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
                cus = prop.multiProcessorCount;
        }
        g_dense_wgs = cus * 4;
    }
    return g_dense_wgs;
}

int g_eval_wgs = 0;     // workgroups of the evaluation grid (0 = one per chunk, capped by ws.nwg)
int g_delta_wgs = 512;  // workgroups of the update grid
int g_moved_share = 64;  // move-driven update when at most this many 1024ths of the vertices moved (< 0: never)
constexpr int MIRROR_WGS = 256;  // workgroups writing mirror bytes after a move-driven update

// Grid of the evaluation for C blocks and nbc batch vertices (every
// workgroup resident at once), and of the single-batch update.
int eval_grid(int C, int nbc, int nwg) {
    const int per_cu = C <= 16 ? eval_wgs_per_cu<16>() : C <= 32 ? eval_wgs_per_cu<32>()
                     : C <= 48 ? eval_wgs_per_cu<48>() : eval_wgs_per_cu<64>();
    const int ch = C <= 16 ? eval_chunk<16>() : C <= 32 ? eval_chunk<32>() : C <= 48 ? eval_chunk<48>() : eval_chunk<64>();
    const int nchunks = (nbc + ch - 1) / ch;
    int grid = nwg / 4 * per_cu;
    if (g_eval_wgs > 0 && grid > g_eval_wgs) grid = g_eval_wgs;
    if (grid > nwg) grid = nwg;
    if (grid > nchunks) grid = nchunks;
    return grid < 1 ? 1 : grid;
}
int update_grid(int n, int nwg) {
    const int cus = nwg / 4 > 0 ? nwg / 4 : 1;
    int ugrid = (n + UPD_GRID_V - 1) / UPD_GRID_V;
    if (ugrid > g_delta_wgs) ugrid = g_delta_wgs;
    if (ugrid > cus) ugrid = cus;
    return ugrid;
}
constexpr int UPDATE_VERTEX_COST = 2;  // a vertex's head work, in edge ends

int dense_build(const GDev &g, DenseBM &bm, int *delta, hipStream_t s) {
    const int CC = g.C * g.C;
    hipLaunchKernelGGL(k_zero, dim3(grid_for(CC, 256, 64)), dim3(256), 0, s, bm.M, CC);
    hipLaunchKernelGGL(k_zero, dim3(grid_for(CC, 256, 64)), dim3(256), 0, s, delta, CC);
    hipLaunchKernelGGL(k_ftab, dim3(grid_for((long long)bm.ftab_max + 1, 256, 8192)), dim3(256), 0, s, bm.ftab,
                       bm.ftab_max);
    hipLaunchKernelGGL(k_dense_hist, dim3(grid_for(g.n, 256, 1024)), dim3(256), 0, s, g, bm.M);
    hipLaunchKernelGGL(k_dense_final, dim3(1), dim3(FIN_T), 0, s, g, bm, delta, (const long long *)nullptr,
                       (const double *)nullptr, 0, (sbp_sweep_stats_dev *)nullptr, (const unsigned char *)nullptr,
                       -1);
    // balanced vertex ranges for the single-batch update grid
    const int gu = update_grid(g.n, dense_workgroups());
    hipLaunchKernelGGL(k_dense_bounds, dim3(grid_for(gu + 1, 256, 16)), dim3(256), 0, s, g,
                       gu <= SBP_DENSE_BOUNDS - 2 ? gu : 0, UPDATE_VERTEX_COST, bm.bounds);
    // mirrors of the edge ends, verified (flags[0] stays 1 only if all match)
    hipLaunchKernelGGL(k_set_flags, dim3(1), dim3(1), 0, s, bm.flags);
    int rc;
    if ((rc = fill_i32(bm.mir_i, -1, g.e, s))) return rc;
    if (g.n > 0)
        hipLaunchKernelGGL(k_dense_mirror, dim3(grid_for((long long)g.n * 64, 256, 4096)), dim3(256), 0, s, g, bm);
    if (g.e > 0) hipLaunchKernelGGL(k_dense_mirror_check, dim3(grid_for(g.e, 256, 4096)), dim3(256), 0, s, bm, g.e);
    SBP_LAUNCH_CHECK();
    return dense_refresh_ends(g, bm, s);
}

int dense_refresh_ends(const GDev &g, DenseBM &bm, hipStream_t s) {
    if (g.n > 0) {
        hipLaunchKernelGGL(k_dense_ends, dim3(grid_for((long long)g.n * 64, 256, 4096)), dim3(256), 0, s, g, bm);
        SBP_LAUNCH_CHECK();
    }
    return 0;
}

template <bool ENDS, bool TRACE, int CM>
void launch_eval(int grid, hipStream_t s, const EvalArgs &a, const SweepTraceDev &tr) {
    ProfileScope prof("sweep_eval", s, true);  // the kernel's own start and stop times
    hipExtLaunchKernelGGL((k_dense_eval<ENDS, TRACE, CM>), dim3(grid), dim3(EVAL_T), 0, s, prof.start, prof.stop, 0,
                          a, tr);
}

// Launches the evaluation for block capacity CM; returns its grid (the number
// of statistics partials it writes).
template <int CM>
int run_eval(const GDev &g, const DenseBM &bm, DenseScratch &ws, const SweepTraceDev &tr, hipStream_t s) {
    EvalArgs a{};
    a.out_ptr = g.out_ptr;
    a.in_ptr = g.in_ptr;
    a.out_idx = g.out_idx;
    a.in_idx = g.in_idx;
    a.lab = g.lab;
    a.M = bm.M;
    a.dout = bm.dout;
    a.din = bm.din;
    a.fM = bm.fM;
    a.ftab = bm.ftab;
    a.nlo = bm.nl;
    a.nli = bm.nl + bm.nl_in;
    a.nb = ws.nb;
    a.hubrank = ws.hubrank;
    a.stats_part = ws.stats_part;
    a.sum_part = ws.sum_part;
    a.seed = g.seed;
    a.beta = g.beta;
    a.ftab_max = bm.ftab_max;
    a.sweep = g.sweep;
    a.sweep_dev = g.sweep_dev;
    a.n = g.n;
    a.C = g.C;
    a.batch = g.batch;
    a.n_batches = g.n_batches;
    a.eps = g.eps;
    a.voff = g.voff;
    const int nbc = (g.n - g.batch + g.n_batches - 1) / g.n_batches;
    const int grid = eval_grid(g.C, nbc, ws.nwg);
    const bool ends = g.n_batches == 1;
    const bool trace = tr.prop || tr.dS || tr.lnH || tr.margin || tr.accept || tr.status;
    if (ends) {
        if (trace) launch_eval<true, true, CM>(grid, s, a, tr);
        else launch_eval<true, false, CM>(grid, s, a, tr);
    } else {
        if (trace) launch_eval<false, true, CM>(grid, s, a, tr);
        else launch_eval<false, false, CM>(grid, s, a, tr);
    }
    return grid;
}

int dense_sweep_batch(const GDev &g, DenseBM &bm, DenseScratch &ws, const SweepTraceDev &tr,
                      sbp_sweep_stats_dev *stats, hipStream_t s) {
    const int nbc = (g.n - g.batch + g.n_batches - 1) / g.n_batches;
    int grid;
    if (g.C <= 16) grid = run_eval<16>(g, bm, ws, tr, s);
    else if (g.C <= 32) grid = run_eval<32>(g, bm, ws, tr, s);
    else if (g.C <= 48) grid = run_eval<48>(g, bm, ws, tr, s);
    else grid = run_eval<64>(g, bm, ws, tr, s);
    if (g.n_batches == 1) {
        // one workgroup per CU; the decisions of the first sl vertices in the
        // LDS the workgroup leaves free
        const int ugrid = update_grid(g.n, ws.nwg);
        const size_t fixed = (sizeof(int) * ((size_t)g.C * g.C + 4 * CHU + 3) + 15) & ~(size_t)15;
        const size_t budget = (size_t)dense_lds_per_block() - 1024;
        size_t sl = budget > fixed ? budget - fixed : 0;
        if (sl > (size_t)g.n) sl = (size_t)g.n;
        sl &= ~(size_t)15;
        const bool vec = ((uintptr_t)g.out_idx % 16 == 0) && ((uintptr_t)g.in_idx % 16 == 0);
        if (ugrid > 0) {
            if (vec)
                hipLaunchKernelGGL(k_dense_update<true>, dim3(ugrid), dim3(UPD_T), fixed + sl, s, g, bm,
                                   (const unsigned char *)ws.nb, ws.delta, (int)sl,
                                   (const long long *)ws.stats_part, grid, g_moved_share);
            else
                hipLaunchKernelGGL(k_dense_update<false>, dim3(ugrid), dim3(UPD_T), fixed + sl, s, g, bm,
                                   (const unsigned char *)ws.nb, ws.delta, (int)sl,
                                   (const long long *)ws.stats_part, grid, g_moved_share);
        }
    } else {
        hipLaunchKernelGGL(k_dense_delta, dim3(grid), dim3(256), 0, s, g, (const int *)ws.nb, ws.delta);
        hipLaunchKernelGGL(k_dense_apply, dim3(grid_for(nbc, 256, 2048)), dim3(256), 0, s, g, (const int *)ws.nb);
    }
    // one batch: workgroups 1.. write the moved vertices' mirror bytes when the
    // update left them (a no-op after a streaming update)
    const bool one = g.n_batches == 1;
    hipLaunchKernelGGL(k_dense_final, dim3(one ? 1 + MIRROR_WGS : 1), dim3(FIN_T), 0, s, g, bm, ws.delta,
                       ws.stats_part, ws.sum_part, grid, stats, one ? (const unsigned char *)ws.nb : nullptr,
                       g.batch == 0 ? ws.hub_slot : -1);
    SBP_LAUNCH_CHECK();
    return 0;
}

// Engine path: one sweep batch of every listed graph on the dense kernels,
// against the union sparse blockmodel built for this step.  Per graph: a dense
// copy of its blockmodel in its slot, then one persistent evaluation launch
// per block-capacity class with a work queue per graph.  Decisions go to each
// job's nb as ints (-1 = stays); the caller applies them.
size_t dense_multi_scratch_bytes(int max_graphs) {
    const size_t G = (size_t)(max_graphs > 0 ? max_graphs : 1);
    return ((G * sizeof(EvalArgs) + 255) & ~(size_t)255) + ((G * sizeof(ToDense) + 255) & ~(size_t)255) +
           3 * ((G * sizeof(int) + 255) & ~(size_t)255) + 256;
}

void fill_ftab(double *tab, unsigned n_max, hipStream_t s) {
    hipLaunchKernelGGL(k_ftab, dim3(grid_for((long long)n_max + 1, 256, 8192)), dim3(256), 0, s, tab, n_max);
}

int dense_multi_sweep(const std::vector<DenseSweepJob> &jobs, const SparseBM &bm, const double *ftab,
                      unsigned ftab_max, void *scratch, int max_graphs, hipStream_t s) {
    const int D = (int)jobs.size();
    if (D == 0) return 0;
    if (D > max_graphs) return fail(-1, "more dense sweeps than the engine's graphs");
    char *b = (char *)scratch;
    const size_t G = (size_t)max_graphs;
    EvalArgs *dA = (EvalArgs *)b;
    b += (G * sizeof(EvalArgs) + 255) & ~(size_t)255;
    ToDense *dJ = (ToDense *)b;
    b += (G * sizeof(ToDense) + 255) & ~(size_t)255;
    int *d_nruns = (int *)b;
    b += (G * sizeof(int) + 255) & ~(size_t)255;
    int *d_gstart = (int *)b;
    b += (G * sizeof(int) + 255) & ~(size_t)255;
    int *d_ctr = (int *)b;
    // jobs ordered by block-capacity class
    std::vector<int> order(D);
    auto cls = [&](int C) { return C <= 16 ? 0 : C <= 32 ? 1 : C <= 48 ? 2 : 3; };
    int pos = 0;
    int cstart[5] = {0, 0, 0, 0, 0};
    for (int c = 0; c < 4; ++c) {
        cstart[c] = pos;
        for (int i = 0; i < D; ++i)
            if (cls(jobs[i].g.C) == c) order[pos++] = i;
    }
    cstart[4] = pos;
    const int chunk_of[4] = {eval_chunk<16>(), eval_chunk<32>(), eval_chunk<48>(), eval_chunk<64>()};
    const int per_cu[4] = {eval_wgs_per_cu<16>(), eval_wgs_per_cu<32>(), eval_wgs_per_cu<48>(), eval_wgs_per_cu<64>()};
    const int cus = dense_workgroups() / 4;
    std::vector<EvalArgs> hA(D);
    std::vector<ToDense> hJ(D);
    std::vector<int> nruns(D), gstart(D);
    int grid[4] = {0, 0, 0, 0}, run_len[4] = {1, 1, 1, 1};
    for (int c = 0; c < 4; ++c) {
        long long total = 0;
        for (int k = cstart[c]; k < cstart[c + 1]; ++k) {
            const GDev &g = jobs[order[k]].g;
            const int nbc = (g.n - g.batch + g.n_batches - 1) / g.n_batches;
            total += (nbc + chunk_of[c] - 1) / chunk_of[c];
        }
        if (total == 0) continue;
        grid[c] = (int)std::min<long long>(total, (long long)cus * per_cu[c]);
        // about four runs per workgroup, so that late workgroups can balance
        run_len[c] = (int)std::max<long long>(1, std::min<long long>(64, total / (4LL * grid[c])));
        long long acc = 0;
        for (int k = cstart[c]; k < cstart[c + 1]; ++k) {
            const GDev &g = jobs[order[k]].g;
            const int nbc = (g.n - g.batch + g.n_batches - 1) / g.n_batches;
            const int nch = (nbc + chunk_of[c] - 1) / chunk_of[c];
            nruns[k] = (nch + run_len[c] - 1) / run_len[c];
            gstart[k] = (int)(acc * grid[c] / total);  // first workgroup of the graph's share
            acc += nch;
        }
    }
    for (int k = 0; k < D; ++k) {
        const DenseSweepJob &j = jobs[order[k]];
        const GDev &g = j.g;
        EvalArgs a{};
        a.out_ptr = g.out_ptr;
        a.in_ptr = g.in_ptr;
        a.out_idx = g.out_idx;
        a.in_idx = g.in_idx;
        a.lab = g.lab;
        a.M = j.M;
        a.dout = j.dout;
        a.din = j.din;
        a.fM = j.fM;
        a.ftab = ftab;
        a.ftab_max = ftab_max;
        a.nb = j.nb;
        a.seed = g.seed;
        a.beta = g.beta;
        a.sweep = g.sweep;
        a.n = g.n;
        a.C = g.C;
        a.batch = g.batch;
        a.n_batches = g.n_batches;
        a.eps = g.eps;
        a.hubrank = g.skip;
        hA[k] = a;
        hJ[k] = ToDense{g.boff, g.C, j.M, j.fM, j.dout, j.din};
    }
    SBP_HIP_CHECK(hipMemcpyAsync(dA, hA.data(), D * sizeof(EvalArgs), hipMemcpyHostToDevice, s));
    SBP_HIP_CHECK(hipMemcpyAsync(dJ, hJ.data(), D * sizeof(ToDense), hipMemcpyHostToDevice, s));
    SBP_HIP_CHECK(hipMemcpyAsync(d_nruns, nruns.data(), D * sizeof(int), hipMemcpyHostToDevice, s));
    SBP_HIP_CHECK(hipMemcpyAsync(d_gstart, gstart.data(), D * sizeof(int), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_to_dense, dim3(D), dim3(256), 0, s, (const ToDense *)dJ, bm, ftab, ftab_max, d_ctr);
    SBP_LAUNCH_CHECK();
    for (int c = 0; c < 4; ++c) {
        const int n = cstart[c + 1] - cstart[c];
        if (n == 0 || grid[c] == 0) continue;
        const int o = cstart[c];
        ProfileScope prof("sweep_eval_multi", s);
        if (c == 0)
            hipLaunchKernelGGL(k_dense_eval_multi<16>, dim3(grid[c]), dim3(EVAL_T), 0, s, (const EvalArgs *)dA + o,
                               (const int *)d_nruns + o, (const int *)d_gstart + o, d_ctr + o, n, run_len[c]);
        else if (c == 1)
            hipLaunchKernelGGL(k_dense_eval_multi<32>, dim3(grid[c]), dim3(EVAL_T), 0, s, (const EvalArgs *)dA + o,
                               (const int *)d_nruns + o, (const int *)d_gstart + o, d_ctr + o, n, run_len[c]);
        else if (c == 2)
            hipLaunchKernelGGL(k_dense_eval_multi<48>, dim3(grid[c]), dim3(EVAL_T), 0, s, (const EvalArgs *)dA + o,
                               (const int *)d_nruns + o, (const int *)d_gstart + o, d_ctr + o, n, run_len[c]);
        else
            hipLaunchKernelGGL(k_dense_eval_multi<64>, dim3(grid[c]), dim3(EVAL_T), 0, s, (const EvalArgs *)dA + o,
                               (const int *)d_nruns + o, (const int *)d_gstart + o, d_ctr + o, n, run_len[c]);
        SBP_LAUNCH_CHECK();
    }
    return 0;
}

int dense_tune(const char *key, long long value) {
    if (!strcmp(key, "dense_eval_workgroups") && value >= 0) {
        g_eval_wgs = (int)value;
        return 0;
    }
    if (!strcmp(key, "dense_update_moved_share") && value >= -1 && value <= 1024) {
        g_moved_share = (int)value;
        return 0;
    }
    if (!strcmp(key, "dense_delta_workgroups") && value >= 1) {
        g_delta_wgs = (int)value;
        return 0;
    }
    return -1;
}

int dense_merge_scores(const GDev &g, const DenseBM &bm, int *partner, double *dS, double *dSl, hipStream_t s) {
    hipLaunchKernelGGL(k_dense_merge, dim3((g.C * 64 + 255) / 256), dim3(256), 0, s, g, bm, partner, dS, dSl);
    SBP_LAUNCH_CHECK();
    return 0;
}


int dense_hub_pass(const GDev &g, DenseBM &bm, DenseScratch &ws, int n_hubs, const HubScratch &h,
                   const SweepTraceDev &tr, hipStream_t s) {
    if (n_hubs <= 0) return 0;
    hipLaunchKernelGGL(k_hub_keys, dim3(grid_for(g.n, 256, 4096)), dim3(256), 0, s, g, h.k0, h.hubrank);
    SBP_LAUNCH_CHECK();
    int rc;
    // stable on the degree bits: ties keep the id order the keys were written in
    if ((rc = radix_sort_bits(h.k0, h.k1, nullptr, nullptr, g.n, 32, 48, h.temp, s))) return rc;
    hipLaunchKernelGGL(k_hub_mark, dim3(1), dim3(MARK_T), 0, s, g, (const uint64_t *)h.k0, n_hubs, h.order,
                       h.hubrank, h.kk, h.hoff);
    hipLaunchKernelGGL(k_hub_codes, dim3(n_hubs), dim3(256), 0, s, g, bm, (const int *)h.order, (const int *)h.kk,
                       (const int *)h.hoff, (const int *)h.hubrank, h.codes, h.mpos);
    hipLaunchKernelGGL(k_dense_hubs, dim3(1), dim3(HUBS_T), 0, s, g, bm, (const int *)h.order, n_hubs,
                       (const int *)h.kk, (const int *)h.hoff, (const int *)h.codes, (const int *)h.mpos,
                       ws.stats_part, ws.sum_part, ws.nwg, tr);
    hipLaunchKernelGGL(k_dense_ends_unmirrored, dim3(grid_for((long long)g.n * 64, 256, 4096)), dim3(256), 0, s, g,
                       bm);
    SBP_LAUNCH_CHECK();
    ws.hubrank = h.hubrank;
    ws.hub_slot = ws.nwg;
    return 0;
}

}  // namespace sbp
