// sbp_sparse.hip -- sparse blockmodel tier over a batch of graphs (gfx950).
//
// The graphs of a step are laid side by side: graph g's blocks occupy union
// ids [boff, boff + C) and its edges union slots [eoff, eoff + e).  The union
// blockmodel is block diagonal, so one build serves every graph, and every
// per-graph result depends only on that graph's data (rows, chunk borders and
// reduction trees are taken relative to the graph's own indices).
//
//   M (Sec. II-A) ......... rows: rptr/rcol/rval, columns: cptr/crow/cval
//                           (the hashmap rows and transpose of Sec. III-A (a,b)
//                           as sorted arrays)
//   proposal tables ....... row t of M + M^T in ascending column with running
//                           sums (scol/scum), so a draw from e_t. is a search
//   DL (Eq. 1, Eq. 2) ..... chunked FP64 reduction per graph
//   sweep (Alg. 2) ........ wave per vertex with <= 256 edge ends, workgroup
//                           per hub; neighbour blocks aggregated by a bitonic
//                           sort (the sparse change vector of Sec. III-A (c))
//   merges (Alg. 1) ....... wave per block for scoring; application as a
//                           parallel greedy union over the candidate
//                           pseudoforest (pointer jumping)
#include <mutex>

#include "sbp_internal.h"

namespace sbp {

namespace {

constexpr int BLK = 256;

// ---------------------------------------------------------------- lookups
__device__ __forceinline__ int row_get(const int *__restrict__ ptr, const int *__restrict__ idx,
                                       const int *__restrict__ val, int a, int b) {
    int lo = ptr[a], hi = ptr[a + 1];
    const int end = hi;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (idx[mid] < b) lo = mid + 1; else hi = mid;
    }
    return (lo < end && idx[lo] == b) ? val[lo] : 0;
}
__device__ __forceinline__ int m_get(const SparseBM &bm, int a, int b) { return row_get(bm.rptr, bm.rcol, bm.rval, a, b); }
__device__ __forceinline__ int mt_get(const SparseBM &bm, int b, int a) { return row_get(bm.cptr, bm.crow, bm.cval, b, a); }

// smallest s whose running sum of e_ts (ascending s) exceeds x, 0 <= x < d_t
__device__ __forceinline__ int s_draw(const SparseBM &bm, int t, long long x) {
    int lo = bm.rptr[t] + bm.cptr[t], hi = bm.rptr[t + 1] + bm.cptr[t + 1];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((long long)bm.scum[mid] <= x) lo = mid + 1; else hi = mid;
    }
    return bm.scol[lo];
}

__device__ __forceinline__ double model_terms(double E, double N, double C) {
    const double c2 = C * C;
    return xlogx(E + c2) - xlogx(E) - xlogx(c2) + N * log(C);
}

// ---------------------------------------------------------------- build
// Workgroup per BLK consecutive union vertices: their union edge ranges and
// source keys go to LDS, then the workgroup's threads take the edges in order,
// each finding its source vertex there, so hubs do not serialise a thread.
__global__ void __launch_bounds__(BLK) k_edge_keys(const GDev *__restrict__ G, const int *__restrict__ vstart,
                                                   int nG, int Ntot, int Ctot, uint64_t *__restrict__ keys) {
    __shared__ long long U[BLK + 1];  // union edge start of each vertex, then the end of the last
    __shared__ uint64_t base[BLK];
    __shared__ int gi[BLK];
    for (int b0 = blockIdx.x * BLK; b0 < Ntot; b0 += gridDim.x * BLK) {
        const int nv = min(BLK, Ntot - b0);
        __syncthreads();  // previous range done with the LDS
        if ((int)threadIdx.x < nv) {
            const int t = threadIdx.x, i = b0 + t;
            const int g = find_graph(vstart, nG, i);
            const GDev &d = G[g];
            const int v = i - d.voff;
            U[t] = d.eoff + d.out_ptr[v];
            base[t] = (uint64_t)(d.boff + d.lab[v]) * (uint64_t)Ctot + (uint64_t)d.boff;
            gi[t] = g;
            if (t == nv - 1) U[nv] = d.eoff + d.out_ptr[v + 1];
        }
        __syncthreads();
        const long long e1 = U[nv];
        for (long long x = U[0] + threadIdx.x; x < e1; x += BLK) {
            int lo = 0, hi = nv - 1;  // last vertex whose range starts at or before x
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (U[mid] <= x) lo = mid; else hi = mid - 1;
            }
            const GDev &d = G[gi[lo]];
            keys[x] = base[lo] + (uint64_t)d.lab[d.out_idx[x - d.eoff]];
        }
    }
}

__global__ void k_rle_flags(const uint64_t *__restrict__ keys, long long n, int *__restrict__ flags) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        flags[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

__global__ void k_rle_emit(const uint64_t *__restrict__ keys, const int *__restrict__ flags,
                           const long long *__restrict__ pos, long long n, int Ctot, int *__restrict__ urow,
                           int *__restrict__ rcol, int *__restrict__ start) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        if (!flags[i]) continue;
        const long long k = pos[i];
        const uint64_t key = keys[i];
        urow[k] = (int)(key / (uint64_t)Ctot);
        rcol[k] = (int)(key % (uint64_t)Ctot);
        start[k] = (int)i;
    }
}

__global__ void k_rle_count(const int *__restrict__ start, const long long *__restrict__ nnz_p, long long n,
                            int *__restrict__ rval) {
    const long long nnz = *nnz_p;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (long long)gridDim.x * blockDim.x)
        rval[k] = (int)((k + 1 < nnz ? (long long)start[k + 1] : n) - start[k]);
}

// ptr[a] = first entry whose key is >= a, for a in [0, C]
__global__ void k_lower_bounds(const int *__restrict__ keys, const long long *__restrict__ nnz_p, int C,
                               int *__restrict__ ptr) {
    const int nnz = (int)*nnz_p;
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a <= C; a += gridDim.x * blockDim.x) {
        int lo = 0, hi = nnz;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (keys[mid] < a) lo = mid + 1; else hi = mid;
        }
        ptr[a] = lo;
    }
}

__global__ void k_csc_keys(const int *__restrict__ urow, const int *__restrict__ rcol, const int *__restrict__ rval,
                           const long long *__restrict__ nnz_p, long long cap, int Ctot, uint64_t *__restrict__ k2,
                           uint64_t *__restrict__ v2) {
    const long long nnz = *nnz_p;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < cap; k += (long long)gridDim.x * blockDim.x) {
        if (k < nnz) {
            k2[k] = (uint64_t)rcol[k];
            v2[k] = ((uint64_t)(uint32_t)urow[k] << 32) | (uint32_t)rval[k];
        } else {
            k2[k] = (uint64_t)Ctot;
            v2[k] = 0;
        }
    }
}

__global__ void k_csc_emit(const uint64_t *__restrict__ k2, const uint64_t *__restrict__ v2,
                           const long long *__restrict__ nnz_p, int *__restrict__ ccol, int *__restrict__ crow,
                           int *__restrict__ cval) {
    const long long nnz = *nnz_p;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (long long)gridDim.x * blockDim.x) {
        ccol[k] = (int)k2[k];
        crow[k] = (int)(v2[k] >> 32);
        cval[k] = (int)(v2[k] & 0xffffffffu);
    }
}

// Wave per block t: degrees, then row t of M + M^T merged in ascending column
// (row entries first on equal columns) with running sums.  When row and
// column together fit the wave, each entry finds its merged position by a
// search of the other list in LDS (row entry i goes to i + #column entries
// below it, column entry j to j + #row entries at or below it); longer blocks
// take 64 merged positions at a time by merge-path searches.
__global__ void __launch_bounds__(BLK) k_block_rows(SparseBM bm) {
    constexpr int NW = BLK / 64;
    __shared__ int SA[NW][64], SB[NW][64], MC[NW][64], MV[NW][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int t = wave; t < bm.Ctot; t += nwaves) {
        const int r0 = bm.rptr[t], lr = bm.rptr[t + 1] - r0;
        const int c0 = bm.cptr[t], lc = bm.cptr[t + 1] - c0;
        const int *A = bm.rcol + r0, *Av = bm.rval + r0;
        const int *B = bm.crow + c0, *Bv = bm.cval + c0;
        const int s0 = r0 + c0, L = lr + lc;
        if (L <= 64) {
            int a = 0, av = 0, b = 0, bv = 0;
            if (lane < lr) {
                a = A[lane];
                av = Av[lane];
            }
            if (lane < lc) {
                b = B[lane];
                bv = Bv[lane];
            }
            const int so = wave_sum_i32(av), si = wave_sum_i32(bv);
            if (lane == 0) {
                bm.dout[t] = so;
                bm.din[t] = si;
            }
            SA[wv][lane] = a;
            SB[wv][lane] = b;
            wave_sync_lds();
            if (lane < lr) {
                int lo = 0, hi = lc;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (SB[wv][mid] < a) lo = mid + 1; else hi = mid;
                }
                MC[wv][lane + lo] = a;
                MV[wv][lane + lo] = av;
            }
            if (lane < lc) {
                int lo = 0, hi = lr;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (SA[wv][mid] <= b) lo = mid + 1; else hi = mid;
                }
                MC[wv][lane + lo] = b;
                MV[wv][lane + lo] = bv;
            }
            wave_sync_lds();
            int x = lane < L ? MV[wv][lane] : 0;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o, SBP_WAVE);
                if (lane >= o) x += y;
            }
            if (lane < L) {
                bm.scol[s0 + lane] = MC[wv][lane];
                bm.scum[s0 + lane] = x;
            }
            wave_sync_lds();
            continue;
        }
        int so = 0, si = 0;
        for (int j = lane; j < lr; j += 64) so += Av[j];
        for (int j = lane; j < lc; j += 64) si += Bv[j];
        so = wave_sum_i32(so);
        si = wave_sum_i32(si);
        if (lane == 0) {
            bm.dout[t] = so;
            bm.din[t] = si;
        }
        int carry = 0;
        for (int base = 0; base < L; base += 64) {
            const int q = base + lane;
            int col = 0, val = 0;
            if (q < L) {
                int lo = q - lc > 0 ? q - lc : 0, hi = q < lr ? q : lr;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (A[mid] <= B[q - 1 - mid]) lo = mid + 1; else hi = mid;
                }
                const int i = lo, j = q - lo;
                if (i < lr && (j >= lc || A[i] <= B[j])) {
                    col = A[i];
                    val = Av[i];
                } else {
                    col = B[j];
                    val = Bv[j];
                }
            }
            int x = val;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o, SBP_WAVE);
                if (lane >= o) x += y;
            }
            if (q < L) {
                bm.scol[s0 + q] = col;
                bm.scum[s0 + q] = carry + x;
            }
            carry += __shfl(x, 63, SBP_WAVE);
        }
    }
}

// ---------------------------------------------------------------- description length
constexpr int DL_CHUNK = 2048;

__global__ void __launch_bounds__(BLK) k_dl_partial(const GDev *__restrict__ G, const int *__restrict__ chstart, int nG,
                                                   int nchunks, SparseBM bm, double *__restrict__ part) {
    __shared__ double ws[BLK / SBP_WAVE];
    const int ch = blockIdx.x;
    if (ch >= nchunks) return;
    const int g = find_graph(chstart, nG, ch);
    const GDev &d = G[g];
    const int local = ch - chstart[g];
    const int nE = (d.e + DL_CHUNK - 1) / DL_CHUNK;
    double acc = 0.0;
    if (local < nE) {
        const int k0 = bm.rptr[d.boff], k1 = bm.rptr[d.boff + d.C];
        for (int i = threadIdx.x; i < DL_CHUNK; i += BLK) {
            const int k = k0 + local * DL_CHUNK + i;
            if (k < k1) acc += xlogx((double)bm.rval[k]);
        }
    } else {
        const int base = (local - nE) * DL_CHUNK;
        for (int i = threadIdx.x; i < DL_CHUNK; i += BLK) {
            const int x = base + i;
            if (x < d.C) acc -= xlogx((double)bm.dout[d.boff + x]);
            else if (x < 2 * d.C) acc -= xlogx((double)bm.din[d.boff + x - d.C]);
        }
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < BLK / SBP_WAVE; ++w) t += ws[w];
        part[ch] = t;
    }
}

// DL of every graph from its chunk partials: a wave per graph, lane l adding
// the graph's partials l, l + 64, ... (counted from the graph's first chunk),
// so the sum does not depend on the other graphs of a batch.
__global__ void __launch_bounds__(64) k_dl_final(const GDev *__restrict__ G, const int *__restrict__ chstart, int nG,
                                                 int nchunks, const double *__restrict__ part,
                                                 double *__restrict__ dl) {
    const int g = blockIdx.x, lane = threadIdx.x;
    if (g >= nG) return;
    const GDev &d = G[g];
    const int c0 = chstart[g], c1 = g + 1 < nG ? chstart[g + 1] : nchunks;
    double L = 0.0;
    for (int c = c0 + lane; c < c1; c += 64) L += part[c];
    L = wave_sum(L);
    if (lane == 0) dl[g] = model_terms((double)d.e, (double)d.n, (double)d.C) - L;
}

// ---------------------------------------------------------------- vertex moves
struct MoveOut {
    int s;  // proposed block (union id)
    double dS, lnH, margin;
    bool accept;
};

__device__ __forceinline__ void record_move(const GDev &d, int v, int r, const MoveOut &o, bool noop, int *nb,
                                            const SweepTraceDev &tr) {
    const int u = d.voff + v;
    const bool acc = !noop && o.accept;
    nb[u] = acc ? o.s - d.boff : -1;
    if (tr.prop) tr.prop[u] = o.s - d.boff;
    if (tr.dS) tr.dS[u] = noop ? 0.0 : o.dS;
    if (tr.lnH) tr.lnH[u] = noop ? 0.0 : o.lnH;
    if (tr.margin) tr.margin[u] = noop ? 0.0 : o.margin;
    if (tr.accept) tr.accept[u] = acc ? 1 : 0;
    // -1 no-op, else accepted (bit 0) and near tie (bit 1)
    if (tr.status) tr.status[u] = noop ? -1 : (acc ? 1 : 0) + (fabs(o.margin) < SBP_NEAR_TIE ? 2 : 0);
}

constexpr int LEAF_WAVES = 4;
constexpr int KEY_PAD = 0x7fffffff;
constexpr int KEY_SELF = 0x7ffffffe;  // self-loop end: after every block key, before the padding

constexpr int SMALL_K = 30;  // vertices with at most this many edge ends go two to eight to a wave

// Whether flat sweep item i is a vertex of the current batch with kmin..kmax
// edge ends.
__device__ __forceinline__ bool sweep_item(const GDev *G, const int *starts, int nG, int n_items, int i, int kmin,
                                           int kmax) {
    if (i >= n_items) return false;
    const int g = find_graph(starts, nG, i);
    const GDev &d = G[g];
    const int v = i - starts[g];
    const int k = d.out_ptr[v + 1] - d.out_ptr[v] + d.in_ptr[v + 1] - d.in_ptr[v];
    return in_batch(d, v) && k >= kmin && k <= kmax;
}

// s_draw by a whole wave over t's running sums [lo, hi): each round probes 64
// evenly spaced sums and keeps the stretch between the last probe at or below
// x and the first above; the probes read their blocks too, so the round that
// probes single entries yields s.
__device__ __forceinline__ int s_draw_wave(const SparseBM &bm, int lo, int hi, long long x) {
    const int lane = threadIdx.x & 63;
    for (;;) {
        const int st = (hi - lo + 63) >> 6;
        const int p = min(lo + (lane + 1) * st, hi) - 1;  // the last probe is hi - 1, whose sum d_t exceeds x
        const int sc = bm.scum[p], sb = bm.scol[p];
        const int f = __builtin_ctzll(__ballot((long long)sc > x));
        if (st == 1) return __shfl(sb, f, 64);
        const int nlo = min(lo + f * st, hi);
        hi = min(lo + (f + 1) * st, hi);
        lo = nlo;
    }
}

// Row r, row s, column r and column s of M for one move: list l holds
// (index, value) pairs ascending by index.  A list of at most ROW entries is
// staged in LDS whole; one of at most ROW * SPAN entries keeps in LDS only
// the last index of every SPAN-entry window (samples, at l * ROW of samp) and
// is otherwise read in place; a longer one is read in place.
constexpr int LEAF_ROW = 128;
constexpr int SPAN = 16;
struct MoveLists {
    const int *c[4], *v[4];
    int n[4];
    const int *samp;  // the samples of the sampled lists
    int sampled;      // bit l: list l is sampled
};

// List l of a move, staged by the calling lanes (lane0 of nl) into sc / sv.
template <int ROW>
__device__ __forceinline__ void stage_list(MoveLists &L, int l, const int *gc, const int *gv, int n, int *sc, int *sv,
                                           int lane0, int nl) {
    L.n[l] = n;
    sc += l * ROW;
    if (n <= ROW) {
        sv += l * ROW;
        for (int j = lane0; j < n; j += nl) {
            sc[j] = gc[j];
            sv[j] = gv[j];
        }
        L.c[l] = sc;
        L.v[l] = sv;
    } else {
        L.c[l] = gc;
        L.v[l] = gv;
        if (n <= ROW * SPAN) {
            const int ns = (n + SPAN - 1) / SPAN;
            for (int i = lane0; i < ns; i += nl) sc[i] = gc[min(SPAN * (i + 1), n) - 1];
            L.sampled |= 1 << l;
        }
    }
}

// The entries at index t of the four lists (0 where absent): lower-bound
// searches by descending powers of two, run side by side so that every step
// issues one load per list and the four share their round trips.  In a
// sampled list every probe of a step of at least SPAN falls on the last entry
// of a window (or on the list's last entry), so it reads the LDS sample.
template <int ROW>
__device__ __forceinline__ void lists_lookup(const MoveLists &L, int nmax, int t, int out[4]) {
    int lo[4] = {0, 0, 0, 0};
    for (int st = nmax > 0 ? 1 << (31 - __clz(nmax)) : 0; st > 0; st >>= 1) {
        int kv[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int i = min(lo[l] + st, L.n[l]) - 1;
            kv[l] = L.n[l] <= 0 ? 0
                    : (st >= SPAN && ((L.sampled >> l) & 1)) ? L.samp[l * ROW + i / SPAN]
                                                              : L.c[l][i];
        }
#pragma unroll
        for (int l = 0; l < 4; ++l)
            if (lo[l] + st <= L.n[l] && kv[l] < t) lo[l] += st;
    }
    int kv[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) kv[l] = lo[l] < L.n[l] ? L.c[l][lo[l]] : -1;
#pragma unroll
    for (int l = 0; l < 4; ++l) out[l] = kv[l] == t ? L.v[l][lo[l]] : 0;
}

// The four entries (M_rt, M_st, M_tr, M_ts) of a move from r to s for the
// neighbour block t (union ids): one load each from the graph's lookup table
// when use_tab (the graph has one and a row or column of r or s is longer
// than the LDS stage), else searches of the staged lists (an LDS search beats
// a table load when the lists fit the stage).
template <int ROW>
__device__ __forceinline__ void entries4(const GDev &d, bool use_tab, const MoveLists &L, int nmax, int r, int s,
                                         int t, int out[4]) {
    if (use_tab) {
        const int C = d.C, rl = r - d.boff, sl = s - d.boff, tl = t - d.boff;
        const int *__restrict__ M = d.mdense;
        out[0] = M[rl * C + tl];
        out[1] = M[sl * C + tl];
        out[2] = M[tl * C + rl];
        out[3] = M[tl * C + sl];
    } else {
        lists_lookup<ROW>(L, nmax, t, out);
    }
}

// f(x) = x ln x of the integers below FT_N, built by each workgroup in LDS
// with the same xlogx as the direct path, so both give identical values.
constexpr int FT_N = 512;
__device__ __forceinline__ void ft_fill(double *ft) {
    for (int x = threadIdx.x; x < FT_N; x += blockDim.x) ft[x] = xlogx((double)x);
    __syncthreads();
}
__device__ __forceinline__ double ftx(const double *ft, int x) {
    return (unsigned)x < (unsigned)FT_N ? ft[x] : xlogx((double)x);
}

// DL and proposal terms of one distinct neighbour block t other than r and
// s: Mv = (M_rt, M_st, M_tr, M_ts), ko / ki the out / in ends of v into t,
// dtt = d_t.
__device__ __forceinline__ void block_terms(const double *ft, int ko, int ki, const int Mv[4], long long dtt,
                                            double eps, double epsC, double &dL, double &qf, double &qr) {
    const int Mrt = Mv[0], Mst = Mv[1], Mtr = Mv[2], Mts = Mv[3];
    if (ko) dL += ftx(ft, Mrt - ko) - ftx(ft, Mrt) + ftx(ft, Mst + ko) - ftx(ft, Mst);
    if (ki) dL += ftx(ft, Mtr - ki) - ftx(ft, Mtr) + ftx(ft, Mts + ki) - ftx(ft, Mts);
    const double kt = (double)(ko + ki);
    const double den = (double)dtt + epsC;
    qf += kt * (((double)(Mts + Mst) + eps) / den);
    qr += kt * (((double)(Mtr - ki + Mrt - ko) + eps) / den);
}

// Term cl of the blocks r and s themselves, one per lane: 0-3 the corner
// entries rr, rs, sr, ss; 4-7 the block degrees (opposite sign); 8-9 the
// forward and 10-11 the reverse proposal weights of r and s.  kpr / kps pack
// v's out | in << 16 ends into r / s.
struct CornerIn {
    int Mrr, Mrs, Msr, Mss, kpr, kps, ell, kout, kin, dor, dos, dir, dis;
};
__device__ __forceinline__ void corner_term(const double *ft, int cl, const CornerIn &c, double eps, double epsC,
                                            double &dL, double &qf, double &qr) {
    const int ko_r = c.kpr & 0xffff, ki_r = c.kpr >> 16, ko_s = c.kps & 0xffff, ki_s = c.kps >> 16;
    const int drr = -ko_r - ki_r - c.ell, drs = -ko_s + ki_r, dsr = ko_r - ki_s, dss = ko_s + ki_s + c.ell;
    if (cl < 8) {
        int x, y;
        switch (cl) {
            case 0: x = c.Mrr + drr, y = c.Mrr; break;
            case 1: x = c.Mrs + drs, y = c.Mrs; break;
            case 2: x = c.Msr + dsr, y = c.Msr; break;
            case 3: x = c.Mss + dss, y = c.Mss; break;
            case 4: x = c.dor - c.kout, y = c.dor; break;
            case 5: x = c.dos + c.kout, y = c.dos; break;
            case 6: x = c.dir - c.kin, y = c.dir; break;
            default: x = c.dis + c.kin, y = c.dis; break;
        }
        const double f = ftx(ft, x) - ftx(ft, y);
        dL += cl < 4 ? f : -f;
    } else if (cl < 12) {
        const double kd = (double)(c.kout + c.kin);
        const double d_r = (double)c.dor + (double)c.dir, d_s = (double)c.dos + (double)c.dis;
        int w, num;
        double den;
        switch (cl) {
            case 8: w = ko_r + ki_r + 2 * c.ell, num = c.Mrs + c.Msr, den = d_r + epsC; break;
            case 9: w = ko_s + ki_s, num = 2 * c.Mss, den = d_s + epsC; break;
            case 10: w = ko_r + ki_r, num = 2 * (c.Mrr + drr), den = d_r - kd + epsC; break;
            default: w = ko_s + ki_s + 2 * c.ell, num = c.Msr + dsr + c.Mrs + drs, den = d_s + kd + epsC; break;
        }
        if (w) {
            const double q = (double)w * (((double)num + eps) / den);
            if (cl < 10) qf += q; else qr += q;
        }
    }
}

// Wave per vertex with at most SBP_LEAF_MAX edge ends.  The edge-end keys are
// gathered first (one to four per lane), so the proposal reads the drawn end's
// block from a register; keys are sorted in registers when they fit one per
// lane.  The distinct neighbour blocks, with r and s always among them, take
// their four M entries from one interleaved search each; the lanes holding r
// and s publish the corner entries, and the corner, degree and Hastings terms
// of r and s are spread over lanes 0..11 before the three wave sums.
__global__ void __launch_bounds__(LEAF_WAVES * 64) __attribute__((amdgpu_waves_per_eu(4))) k_sweep_leaf(const GDev *__restrict__ G, const int *__restrict__ starts,
                                                               int nG, int n_items, SparseBM bm, int *__restrict__ nb,
                                                               SweepTraceDev tr) {
    __shared__ int K[LEAF_WAVES][SBP_LEAF_MAX];
    __shared__ int Dt[LEAF_WAVES][SBP_LEAF_MAX], PE[LEAF_WAVES][SBP_LEAF_MAX + 1];
    __shared__ int SC[LEAF_WAVES][4 * LEAF_ROW], SV[LEAF_WAVES][4 * LEAF_ROW];
    __shared__ int CV[LEAF_WAVES][8];
    __shared__ double FT[FT_N];
    ft_fill(FT);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int gw = __builtin_amdgcn_readfirstlane(blockIdx.x * LEAF_WAVES + wv), nw = gridDim.x * LEAF_WAVES;
    int *Kw = K[wv];
    const uint64_t below = lanemask_lt();
    for (int tile = gw * 64; tile < n_items; tile += nw * 64) {
        const uint64_t mine = __ballot(sweep_item(G, starts, nG, n_items, tile + lane, SMALL_K + 1, SBP_LEAF_MAX));
        for (uint64_t todo = mine; todo; todo &= todo - 1) {
            const int item = tile + __builtin_ctzll(todo);
            const int g = find_graph(starts, nG, item);
            const GDev &d = G[g];
            const int v = item - starts[g];
            const int op = d.out_ptr[v], kout = d.out_ptr[v + 1] - op;
            const int ip = d.in_ptr[v], kin = d.in_ptr[v + 1] - ip;
            const int k = kout + kin;
            const int r = d.boff + d.lab[v];
            const int rb0 = bm.rptr[r], rb1 = bm.rptr[r + 1], cb0 = bm.cptr[r], cb1 = bm.cptr[r + 1];
            // edge-end keys 2 t + (1 for an in-end), in canonical end order
            int key_c[4];
            int ell = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int j = 64 * c + lane;
                int key = KEY_PAD;
                if (j < k) {
                    const int u = j < kout ? d.out_idx[op + j] : d.in_idx[ip + j - kout];
                    if (u == v) {
                        key = KEY_SELF;
                        if (j < kout) ++ell;
                    } else {
                        key = 2 * (d.boff + d.lab[u]) + (j < kout ? 0 : 1);
                    }
                }
                key_c[c] = key;
            }
            // row r and column r of M, staged while the proposal is drawn
            MoveLists ML;
            ML.samp = SC[wv];
            ML.sampled = 0;
            ML.n[0] = ML.n[1] = ML.n[2] = ML.n[3] = 0;
            const bool rlong = rb1 - rb0 > LEAF_ROW || cb1 - cb0 > LEAF_ROW;
            if (!(d.mdense && rlong)) {  // long lists of a graph with a table are not staged
                stage_list<LEAF_ROW>(ML, 0, bm.rcol + rb0, bm.rval + rb0, rb1 - rb0, SC[wv], SV[wv], lane, 64);
                stage_list<LEAF_ROW>(ML, 2, bm.crow + cb0, bm.cval + cb0, cb1 - cb0, SC[wv], SV[wv], lane, 64);
            }
            const int dor = bm.dout[r], dir = bm.din[r];
            // proposal: the drawn end's block comes from the lane holding its key
            const Words4 W = draw_words(d.seed, (uint32_t)v, d.sweep, 0u, 0u);
            const double lnu = log(draw_unit(W.w[3]));
            int s;
            {
                const long long eC = (long long)d.eps * d.C;
                if (k == 0) {
                    s = d.boff + (int)draw_idx(W.w[2], (uint64_t)d.C);
                } else {
                    const int j = __builtin_amdgcn_readfirstlane((int)draw_idx(W.w[0], (uint64_t)k));
                    const int c = j >> 6;
                    const int kc = c == 0 ? key_c[0] : c == 1 ? key_c[1] : c == 2 ? key_c[2] : key_c[3];
                    const int kj = __builtin_amdgcn_readlane(kc, j & 63);
                    const int t = kj == KEY_SELF ? r : kj >> 1;
                    const long long dt = (long long)bm.dout[t] + bm.din[t];
                    const int p0 = bm.rptr[t] + bm.cptr[t], p1 = bm.rptr[t + 1] + bm.cptr[t + 1];
                    if (draw_idx(W.w[1], (uint64_t)(dt + eC)) < eC) s = d.boff + (int)draw_idx(W.w[2], (uint64_t)d.C);
                    else s = s_draw_wave(bm, p0, p1, draw_idx(W.w[2], (uint64_t)dt));
                }
            }
            if (s == r) {
                MoveOut o;
                o.s = s;
                if (lane == 0) record_move(d, v, r, o, true, nb, tr);
                continue;
            }
            // row s and column s of M
            bool use_tab;
            {
                const int rs0 = bm.rptr[s], rs1 = bm.rptr[s + 1], cs0 = bm.cptr[s], cs1 = bm.cptr[s + 1];
                use_tab = d.mdense && (rlong || rs1 - rs0 > LEAF_ROW || cs1 - cs0 > LEAF_ROW);
                if (!use_tab) {
                    stage_list<LEAF_ROW>(ML, 1, bm.rcol + rs0, bm.rval + rs0, rs1 - rs0, SC[wv], SV[wv], lane, 64);
                    stage_list<LEAF_ROW>(ML, 3, bm.crow + cs0, bm.cval + cs0, cs1 - cs0, SC[wv], SV[wv], lane, 64);
                }
            }
            const int dos = bm.dout[s], dis = bm.din[s];
            ell = wave_sum_i32(ell);
            // sort: bitonic in registers up to 64 keys, else in LDS
            int m = 2;
            while (m < k) m <<= 1;
            if (k <= 64) {
                int key = key_c[0];
                for (int size = 2; size <= m; size <<= 1)
                    for (int stride = size >> 1; stride > 0; stride >>= 1) {
                        const int o = __shfl_xor(key, stride, 64);
                        key = (((lane & size) == 0) == ((lane & stride) == 0)) ? min(key, o) : max(key, o);
                    }
                Kw[lane] = key;
                wave_sync_lds();
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (64 * c + lane < m) Kw[64 * c + lane] = key_c[c];
                wave_sync_lds();
                for (int size = 2; size <= m; size <<= 1) {
                    for (int stride = size >> 1; stride > 0; stride >>= 1) {
                        for (int q = lane; q < (m >> 1); q += 64) {
                            const int i = 2 * stride * (q / stride) + (q % stride), j = i + stride;
                            const bool asc = (i & size) == 0;
                            const int a = Kw[i], b = Kw[j];
                            if ((a > b) == asc) {
                                Kw[i] = b;
                                Kw[j] = a;
                            }
                        }
                        wave_sync_lds();
                    }
                }
            }
            // runs of equal blocks: each run start records its block, its position
            // and the out-ends before it, so a run's counts are differences of
            // consecutive starts; the end of the block keys closes the last run
            const int kk = k - 2 * ell;
            uint64_t hr = 0, hs = 0;
            int D = 0, E = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int p = 64 * c + lane;
                const int key = p < kk ? Kw[p] : KEY_PAD;
                const int prev = (p > 0 && p < kk) ? Kw[p - 1] : -2;
                const bool st = p < kk && (p == 0 || (key >> 1) != (prev >> 1));
                const uint64_t sm = __ballot(st), em = __ballot(p < kk && !(key & 1));
                hr |= __ballot(st && (key >> 1) == r);
                hs |= __ballot(st && (key >> 1) == s);
                if (st) {
                    const int idx = D + __popcll(sm & below);
                    Dt[wv][idx] = key >> 1;
                    PE[wv][idx] = p | (E + __popcll(em & below)) << 16;
                }
                D += __popcll(sm);
                E += __popcll(em);
            }
            if (lane == 0) PE[wv][D] = kk | (kout - ell) << 16;
            // r and s join the items when no edge end of v points there
            const int Dx = D + (hr ? 0 : 1) + (hs ? 0 : 1);
            wave_sync_lds();
            // per distinct block t: the four entries, then its terms
            const double eps = (double)d.eps;
            const double epsC = (double)d.eps * (double)d.C;
            const int nmax = max(max(ML.n[0], ML.n[1]), max(ML.n[2], ML.n[3]));
            double dL = 0.0, qf = 0.0, qr = 0.0;
            for (int i = lane; i < Dx; i += 64) {
                int t, ko = 0, ki = 0;
                if (i < D) {
                    const int a0 = PE[wv][i], a1 = PE[wv][i + 1];
                    t = Dt[wv][i];
                    ko = (a1 >> 16) - (a0 >> 16);
                    ki = ((a1 & 0xffff) - (a0 & 0xffff)) - ko;
                } else {
                    t = (i == D && !hr) ? r : s;
                }
                const int kp = ko | ki << 16;
                const long long dtt = (long long)bm.dout[t] + bm.din[t];
                int Mv[4];
                entries4<LEAF_ROW>(d, use_tab, ML, nmax, r, s, t, Mv);
                if (t == r) {
                    CV[wv][0] = Mv[0];  // M_rr
                    CV[wv][1] = Mv[1];  // M_sr
                    CV[wv][2] = Mv[3];  // M_rs
                    CV[wv][3] = kp;
                } else if (t == s) {
                    CV[wv][4] = Mv[1];  // M_ss
                    CV[wv][5] = kp;
                } else {
                    block_terms(FT, ko, ki, Mv, dtt, eps, epsC, dL, qf, qr);
                }
            }
            wave_sync_lds();
            {
                const CornerIn c{CV[wv][0], CV[wv][2], CV[wv][1], CV[wv][4], CV[wv][3], CV[wv][5], ell, kout, kin,
                                 dor, dos, dir, dis};
                corner_term(FT, lane, c, eps, epsC, dL, qf, qr);
            }
            dL = wave_sum(dL);
            qf = wave_sum(qf);
            qr = wave_sum(qr);
            MoveOut o;
            o.s = s;
            o.dS = -dL;
            o.lnH = k > 0 ? log(qr) - log(qf) : 0.0;
            const double z = -d.beta * o.dS + o.lnH;
            o.margin = z - lnu;
            o.accept = lnu < z;
            if (lane == 0) record_move(d, v, r, o, false, nb, tr);
            wave_sync_lds();
        }
    }
}

constexpr int SMALL_WAVES = 4;
constexpr int SMALL_ROW = 32;  // list entries staged per group

// 64 / GS vertices per wave, a GS-lane group each with one edge end per lane:
// GS = 8 takes the vertices with at most 6 edge ends, GS = 16 those with 7 to
// 14 and GS = 32 those with 15 to 30, so the distinct blocks plus r and s
// never exceed the group and each lane scores one item.  The steps of the wave kernel with group-wide ballots, a GS-way proposal
// search run by all drawing groups together, a GS-lane bitonic sort and DPP
// group sums.  A group left without a vertex in the last round of a tile
// repeats group 0's and records nothing.
template <int GS>
__global__ void __launch_bounds__(SMALL_WAVES * 64) __attribute__((amdgpu_waves_per_eu(GS == 8 ? 4 : 3))) k_sweep_small(const GDev *__restrict__ G,
                                                                 const int *__restrict__ starts, int nG, int n_items,
                                                                 SparseBM bm, int *__restrict__ nb, SweepTraceDev tr) {
    constexpr int NGRP = 64 / GS, KMIN = GS == 8 ? 0 : GS / 2 - 1, KMAX = GS - 2;
    __shared__ int SC[SMALL_WAVES * NGRP][4 * SMALL_ROW], SV[SMALL_WAVES * NGRP][4 * SMALL_ROW];
    __shared__ int Dt[SMALL_WAVES * NGRP][GS], PE[SMALL_WAVES * NGRP][GS + 1];
    __shared__ int CV[SMALL_WAVES * NGRP][8];
    __shared__ double FT[FT_N];
    ft_fill(FT);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, gi = lane / GS, gl = lane % GS;
    const int gs = NGRP * wv + gi;  // the group's LDS slot
    const int sh = GS * gi;
    const uint64_t gm = ((1ull << GS) - 1) << sh, gbelow = lanemask_lt() & gm;
    const int gw = __builtin_amdgcn_readfirstlane(blockIdx.x * SMALL_WAVES + wv), nw = gridDim.x * SMALL_WAVES;
    for (int tile = gw * 64; tile < n_items; tile += nw * 64) {
        // every lane reads its own item's vertex, ends and block-r bounds once
        // per tile; the groups take them from that lane
        int tg = 0, tv = 0, top = 0, tko = 0, tip = 0, tki = 0, tr0 = 0, trp0 = 0, trp1 = 0, tcp0 = 0, tcp1 = 0;
        bool tsmall = false;
        {
            const int it = tile + lane;
            if (it < n_items) {
                tg = find_graph(starts, nG, it);
                const GDev &d = G[tg];
                tv = it - starts[tg];
                top = d.out_ptr[tv];
                tko = d.out_ptr[tv + 1] - top;
                tip = d.in_ptr[tv];
                tki = d.in_ptr[tv + 1] - tip;
                tsmall = in_batch(d, tv) && tko + tki >= KMIN && tko + tki <= KMAX;
                if (tsmall) {
                    tr0 = d.boff + d.lab[tv];
                    trp0 = bm.rptr[tr0];
                    trp1 = bm.rptr[tr0 + 1];
                    tcp0 = bm.cptr[tr0];
                    tcp1 = bm.cptr[tr0 + 1];
                }
            }
        }
        uint64_t todo = __ballot(tsmall);
        while (todo) {
            int mine = -1, first = 0;
#pragma unroll
            for (int q = 0; q < NGRP; ++q) {
                const int pq = todo ? __builtin_ctzll(todo) : -1;
                todo &= todo - 1;
                if (q == 0) first = pq;
                if (q == gi) mine = pq;
            }
            const bool act = mine >= 0;
            const int src = act ? mine : first;
            const int g = __shfl(tg, src, 64), v = __shfl(tv, src, 64);
            const int op = __shfl(top, src, 64), kout = __shfl(tko, src, 64);
            const int ip = __shfl(tip, src, 64), kin = __shfl(tki, src, 64);
            const int r = __shfl(tr0, src, 64);
            const int b0r = __shfl(trp0, src, 64), b1r = __shfl(trp1, src, 64);
            const int c0r = __shfl(tcp0, src, 64), c1r = __shfl(tcp1, src, 64);
            const GDev &d = G[g];
            const int k = kout + kin;
            // the edge end of this lane: key 2 t + (1 for an in-end)
            int key = KEY_PAD, ell = 0;
            if (gl < k) {
                const int u = gl < kout ? d.out_idx[op + gl] : d.in_idx[ip + gl - kout];
                if (u == v) {
                    key = KEY_SELF;
                    ell = gl < kout ? 1 : 0;
                } else {
                    key = 2 * (d.boff + d.lab[u]) + (gl < kout ? 0 : 1);
                }
            }
            // row r and column r of M, staged while the proposal is drawn
            MoveLists ML;
            ML.samp = SC[gs];
            ML.sampled = 0;
            ML.n[0] = ML.n[1] = ML.n[2] = ML.n[3] = 0;
            const bool rlong = b1r - b0r > SMALL_ROW || c1r - c0r > SMALL_ROW;
            if (!(d.mdense && rlong)) {  // long lists of a graph with a table are not staged
                stage_list<SMALL_ROW>(ML, 0, bm.rcol + b0r, bm.rval + b0r, b1r - b0r, SC[gs], SV[gs], gl, GS);
                stage_list<SMALL_ROW>(ML, 2, bm.crow + c0r, bm.cval + c0r, c1r - c0r, SC[gs], SV[gs], gl, GS);
            }
            const int dor = bm.dout[r], dir = bm.din[r];
            // proposal; t's degree and running-sum range come in one round trip
            const Words4 W = draw_words(d.seed, (uint32_t)v, d.sweep, 0u, 0u);
            const double lnu = log(draw_unit(W.w[3]));
            int s = 0;
            long long x = -1;  // draw into t's running sums, or -1
            int lo = 0, hi = 1;
            if (k == 0) {
                s = d.boff + (int)draw_idx(W.w[2], (uint64_t)d.C);
            } else {
                const int kj = __shfl(key, sh + (int)draw_idx(W.w[0], (uint64_t)k), 64);
                const int t = kj == KEY_SELF ? r : kj >> 1;
                const long long eC = (long long)d.eps * d.C;
                const int do_t = bm.dout[t], di_t = bm.din[t];
                const int p0 = bm.rptr[t] + bm.cptr[t], p1 = bm.rptr[t + 1] + bm.cptr[t + 1];
                const long long dt = (long long)do_t + di_t;
                if (draw_idx(W.w[1], (uint64_t)(dt + eC)) < eC) {
                    s = d.boff + (int)draw_idx(W.w[2], (uint64_t)d.C);
                } else {
                    x = draw_idx(W.w[2], (uint64_t)dt);
                    lo = p0;
                    hi = p1;
                }
            }
            // GS-way search of t's running sums by all drawing groups together;
            // each probe also reads its block, so the last round yields s
            {
                bool done = x < 0;
                while (__ballot(!done)) {
                    const int st = (hi - lo + GS - 1) / GS;
                    const int p = min(lo + (gl + 1) * st, hi) - 1;  // the last probe is hi - 1, whose sum exceeds x
                    int sc = 0, sb = 0;
                    if (!done) {
                        sc = bm.scum[p];
                        sb = bm.scol[p];
                    }
                    const bool above = !done && (long long)sc > x;
                    const int f = __builtin_ctzll((__ballot(above) & gm) >> sh | 1ull << GS);
                    const int sf = __shfl(sb, sh + (f & (GS - 1)), 64);
                    if (!done) {
                        if (st == 1) {
                            s = sf;
                            done = true;
                        } else {
                            const int nlo = min(lo + f * st, hi);
                            hi = min(lo + (f + 1) * st, hi);
                            lo = nlo;
                        }
                    }
                }
            }
            const bool live = act && s != r;
            if (act && !live && gl == 0) {
                MoveOut o;
                o.s = s;
                record_move(d, v, r, o, true, nb, tr);
            }
            // row s and column s of M
            bool use_tab;
            {
                const int rs0 = bm.rptr[s], rs1 = bm.rptr[s + 1], cs0 = bm.cptr[s], cs1 = bm.cptr[s + 1];
                use_tab = d.mdense && (rlong || rs1 - rs0 > SMALL_ROW || cs1 - cs0 > SMALL_ROW);
                if (!use_tab) {
                    stage_list<SMALL_ROW>(ML, 1, bm.rcol + rs0, bm.rval + rs0, rs1 - rs0, SC[gs], SV[gs], gl, GS);
                    stage_list<SMALL_ROW>(ML, 3, bm.crow + cs0, bm.cval + cs0, cs1 - cs0, SC[gs], SV[gs], gl, GS);
                }
            }
            const int dos = bm.dout[s], dis = bm.din[s];
            ell = grp_sum_i32<GS>(ell);
            // GS-lane bitonic sort of the group's keys
#pragma unroll
            for (int size = 2; size <= GS; size <<= 1)
#pragma unroll
                for (int stride = size >> 1; stride > 0; stride >>= 1) {
                    const int o = __shfl_xor(key, stride, 64);
                    key = (((gl & size) == 0) == ((gl & stride) == 0)) ? min(key, o) : max(key, o);
                }
            // runs of equal blocks, recorded as in the wave kernel
            const int kk = k - 2 * ell;
            const int prev = __shfl_up(key, 1, GS);
            const bool st = gl < kk && (gl == 0 || (key >> 1) != (prev >> 1));
            const uint64_t sm = __ballot(st) & gm, em = __ballot(gl < kk && !(key & 1)) & gm;
            const bool hr = (__ballot(st && (key >> 1) == r) & gm) != 0;
            const bool hs = (__ballot(st && (key >> 1) == s) & gm) != 0;
            const int D = __popcll(sm);
            if (st) {
                const int idx = __popcll(sm & gbelow);
                Dt[gs][idx] = key >> 1;
                PE[gs][idx] = gl | __popcll(em & gbelow) << 16;
            }
            if (gl == 0) PE[gs][D] = kk | (kout - ell) << 16;
            const int Dx = D + (hr ? 0 : 1) + (hs ? 0 : 1);
            wave_sync_lds();
            const double eps = (double)d.eps;
            const double epsC = (double)d.eps * (double)d.C;
            const int nmax = max(max(ML.n[0], ML.n[1]), max(ML.n[2], ML.n[3]));
            double dL = 0.0, qf = 0.0, qr = 0.0;
            for (int i = gl; i < Dx; i += GS) {
                int tt, ko = 0, ki = 0;
                if (i < D) {
                    const int a0 = PE[gs][i], a1 = PE[gs][i + 1];
                    tt = Dt[gs][i];
                    ko = (a1 >> 16) - (a0 >> 16);
                    ki = ((a1 & 0xffff) - (a0 & 0xffff)) - ko;
                } else {
                    tt = (i == D && !hr) ? r : s;
                }
                const long long dtt = (long long)bm.dout[tt] + bm.din[tt];
                int Mv[4];
                entries4<SMALL_ROW>(d, use_tab, ML, nmax, r, s, tt, Mv);
                if (tt == r) {
                    CV[gs][0] = Mv[0];  // M_rr
                    CV[gs][1] = Mv[1];  // M_sr
                    CV[gs][2] = Mv[3];  // M_rs
                    CV[gs][3] = ko | ki << 16;
                } else if (tt == s) {
                    CV[gs][4] = Mv[1];  // M_ss
                    CV[gs][5] = ko | ki << 16;
                } else {
                    block_terms(FT, ko, ki, Mv, dtt, eps, epsC, dL, qf, qr);
                }
            }
            wave_sync_lds();
            {
                const CornerIn c{CV[gs][0], CV[gs][2], CV[gs][1], CV[gs][4], CV[gs][3], CV[gs][5], ell, kout, kin,
                                 dor, dos, dir, dis};
                for (int cl = gl; cl < 12; cl += GS) corner_term(FT, cl, c, eps, epsC, dL, qf, qr);
            }
            dL = grp_sum<GS>(dL);
            qf = grp_sum<GS>(qf);
            qr = grp_sum<GS>(qr);
            MoveOut o;
            o.s = s;
            o.dS = -dL;
            o.lnH = k > 0 ? log(qr) - log(qf) : 0.0;
            const double z = -d.beta * o.dS + o.lnH;
            o.margin = z - lnu;
            o.accept = lnu < z;
            if (live && gl == 0) record_move(d, v, r, o, false, nb, tr);
            wave_sync_lds();
        }
    }
}

// Workgroup per hub (more than 256 edge ends): keys sorted in global scratch.
constexpr int HUB_THREADS = 512;
constexpr size_t HUB_SLOT_INTS = 4 * (size_t)SBP_MAX_DEGREE_DEV;
constexpr int HUB_LDS = 8192;  // hubs with at most this many sort keys work in LDS

// Per-workgroup LDS of the hub kernel besides the sort and item arrays.
struct HubShared {
    double ft[FT_N];
    double red_d[3 * (HUB_THREADS / 64)];
    int cnt_s[HUB_THREADS / 64], cnt_e[HUB_THREADS / 64], flg[HUB_THREADS / 64];
    int red[HUB_THREADS / 64];
    int cv[6];  // M_rr, M_sr, M_rs, M_ss, then v's packed out | in << 16 ends into r and s
};

// One hub v moving r -> s.  K (kcap ints) first holds the sort keys
// (2 * neighbour block + in-end flag; self-loop ends and padding after them),
// sorted by a bitonic network; the workgroup then records the runs of equal
// block (block in Dt, start position and out-ends before it in PE) and reuses
// K for the M entries of the items: each entry of row r, row s, column r and
// column s finds its index among the sorted items by a binary search and
// stores its value there (as many lists as K has room for; the rest are
// searched per item), catching the corner entries on the way.  Partial sums
// are reduced per wave and then in wave order, so the result does not depend
// on timing.
__device__ __forceinline__ void hub_move(const GDev &d, const SparseBM &bm, int v, int r, int s, int op, int kout,
                                         int ip, int kin, int m, int kcap, double lnu, int *K, int *Dt, int *PE,
                                         int *nb, const SweepTraceDev &tr, HubShared &H) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint64_t below = lanemask_lt();
    const int k = kout + kin;
    int ell = 0;
    for (int j = tid; j < m; j += HUB_THREADS) {
        int key = KEY_PAD;
        if (j < k) {
            const int u = j < kout ? d.out_idx[op + j] : d.in_idx[ip + j - kout];
            if (u == v) {
                key = KEY_SELF;
                if (j < kout) ++ell;
            } else {
                key = 2 * (d.boff + d.lab[u]) + (j < kout ? 0 : 1);
            }
        }
        K[j] = key;
    }
    ell = wave_sum_i32(ell);
    if (lane == 0) H.red[wv] = ell;
    if (tid < 6) H.cv[tid] = 0;
    for (int size = 2; size <= m; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int q = tid; q < (m >> 1); q += HUB_THREADS) {
                const int i = 2 * stride * (q / stride) + (q % stride), j = i + stride;
                const bool asc = (i & size) == 0;
                const int a = K[i], b = K[j];
                if ((a > b) == asc) {
                    K[i] = b;
                    K[j] = a;
                }
            }
        }
    }
    __syncthreads();
    ell = 0;
    for (int w = 0; w < HUB_THREADS / 64; ++w) ell += H.red[w];
    const int kk = k - 2 * ell;
    // runs, HUB_THREADS positions at a time
    int D = 0, E = 0, fl = 0;
    for (int base = 0; base < kk; base += HUB_THREADS) {
        const int p = base + tid;
        const int key = p < kk ? K[p] : KEY_PAD;
        const int prev = (p > 0 && p < kk) ? K[p - 1] : -2;
        const bool st = p < kk && (p == 0 || (key >> 1) != (prev >> 1));
        const uint64_t sm = __ballot(st), em = __ballot(p < kk && !(key & 1));
        const bool fr = __ballot(st && (key >> 1) == r) != 0, fs = __ballot(st && (key >> 1) == s) != 0;
        if (lane == 0) {
            H.cnt_s[wv] = __popcll(sm);
            H.cnt_e[wv] = __popcll(em);
            H.flg[wv] = (fr ? 1 : 0) | (fs ? 2 : 0);
        }
        __syncthreads();
        int ps = D, pe = E;
        for (int w = 0; w < HUB_THREADS / 64; ++w) {
            if (w < wv) {
                ps += H.cnt_s[w];
                pe += H.cnt_e[w];
            }
            D += H.cnt_s[w];
            E += H.cnt_e[w];
            fl |= H.flg[w];
        }
        if (st) {
            const int idx = ps + __popcll(sm & below);
            Dt[idx] = key >> 1;
            PE[idx] = p | (pe + __popcll(em & below)) << 16;
        }
        __syncthreads();
    }
    if (tid == 0) PE[D] = kk | (kout - ell) << 16;
    const bool hr = (fl & 1) != 0, hs = (fl & 2) != 0;
    const int Dx = D + (hr ? 0 : 1) + (hs ? 0 : 1);
    // M entries of the items: the lists that fit in K are joined, the others searched
    MoveLists ML;
    ML.samp = nullptr;
    ML.sampled = 0;
    {
        const int b0[4] = {bm.rptr[r], bm.rptr[s], bm.cptr[r], bm.cptr[s]};
        const int b1[4] = {bm.rptr[r + 1], bm.rptr[s + 1], bm.cptr[r + 1], bm.cptr[s + 1]};
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            ML.c[l] = (l < 2 ? bm.rcol : bm.crow) + b0[l];
            ML.v[l] = (l < 2 ? bm.rval : bm.cval) + b0[l];
            ML.n[l] = b1[l] - b0[l];
        }
    }
    const int nA = min(4, kcap / max(D, 1));
    for (int i = tid; i < nA * D; i += HUB_THREADS) K[i] = 0;
    __syncthreads();
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        if (l >= nA) break;
        for (int j = tid; j < ML.n[l]; j += HUB_THREADS) {
            const int c = ML.c[l][j], val = ML.v[l][j];
            int lo = 0;
            for (int st = D > 0 ? 1 << (31 - __clz(D)) : 0; st > 0; st >>= 1)
                if (lo + st <= D && Dt[lo + st - 1] < c) lo += st;
            if (lo < D && Dt[lo] == c) K[l * D + lo] = val;
            if (l < 2) {
                if (c == r) H.cv[l] = val;      // M_rr from row r, M_sr from row s
                if (c == s) H.cv[2 + l] = val;  // M_rs from row r, M_ss from row s
            }
        }
    }
    MoveLists MS = ML;  // the lists left to search
#pragma unroll
    for (int l = 0; l < 4; ++l)
        if (l < nA) MS.n[l] = 0;
    const int nmax = max(max(MS.n[0], MS.n[1]), max(MS.n[2], MS.n[3]));
    __syncthreads();
    const double eps = (double)d.eps;
    const double epsC = (double)d.eps * (double)d.C;
    double dL = 0.0, qf = 0.0, qr = 0.0;
    for (int i = tid; i < Dx; i += HUB_THREADS) {
        int t, ko = 0, ki = 0;
        if (i < D) {
            const int a0 = PE[i], a1 = PE[i + 1];
            t = Dt[i];
            ko = (a1 >> 16) - (a0 >> 16);
            ki = ((a1 & 0xffff) - (a0 & 0xffff)) - ko;
        } else {
            t = (i == D && !hr) ? r : s;
        }
        const bool corner = t == r || t == s;
        if (corner) H.cv[t == r ? 4 : 5] = ko | ki << 16;
        if (corner && nA >= 2) continue;  // the corner entries came with the joins
        int Mv[4];
        if (corner) {
            MoveLists MA = ML;
            lists_lookup<LEAF_ROW>(MA, max(max(ML.n[0], ML.n[1]), max(ML.n[2], ML.n[3])), t, Mv);
            if (t == r) {
                H.cv[0] = Mv[0];
                H.cv[1] = Mv[1];
            } else {
                H.cv[2] = Mv[0];
                H.cv[3] = Mv[1];
            }
            continue;
        }
        const long long dtt = (long long)bm.dout[t] + bm.din[t];
        lists_lookup<LEAF_ROW>(MS, nmax, t, Mv);
#pragma unroll
        for (int l = 0; l < 4; ++l)
            if (l < nA) Mv[l] = K[l * D + i];
        block_terms(H.ft, ko, ki, Mv, dtt, eps, epsC, dL, qf, qr);
    }
    __syncthreads();
    if (tid < 12) {
        const CornerIn c{H.cv[0], H.cv[2], H.cv[1], H.cv[3], H.cv[4], H.cv[5], ell, kout, kin,
                         bm.dout[r], bm.dout[s], bm.din[r], bm.din[s]};
        corner_term(H.ft, tid, c, eps, epsC, dL, qf, qr);
    }
    dL = wave_sum(dL);
    qf = wave_sum(qf);
    qr = wave_sum(qr);
    if (lane == 0) {
        H.red_d[3 * wv + 0] = dL;
        H.red_d[3 * wv + 1] = qf;
        H.red_d[3 * wv + 2] = qr;
    }
    __syncthreads();
    if (tid == 0) {
        dL = qf = qr = 0.0;
        for (int w = 0; w < HUB_THREADS / 64; ++w) {
            dL += H.red_d[3 * w + 0];
            qf += H.red_d[3 * w + 1];
            qr += H.red_d[3 * w + 2];
        }
        MoveOut o;
        o.s = s;
        o.dS = -dL;
        o.lnH = k > 0 ? log(qr) - log(qf) : 0.0;
        const double z = -d.beta * o.dS + o.lnH;
        o.margin = z - lnu;
        o.accept = lnu < z;
        record_move(d, v, r, o, false, nb, tr);
    }
}

// Sweep evaluation of hub vertices (more than SBP_LEAF_MAX edge ends): a
// workgroup per hub, in LDS up to HUB_LDS sort keys, else in its global slot.
__global__ void __launch_bounds__(HUB_THREADS) k_sweep_hub(const GDev *__restrict__ G, const int *__restrict__ starts,
                                                           int nG, int n_items, SparseBM bm, int *__restrict__ nb,
                                                           SweepTraceDev tr, int *__restrict__ scratch) {
    __shared__ int Ks[HUB_LDS], Dts[HUB_LDS], PEs[HUB_LDS + 1];
    __shared__ HubShared H;
    ft_fill(H.ft);
    int *Kg = scratch + (size_t)blockIdx.x * HUB_SLOT_INTS;
    int *Dtg = Kg + SBP_MAX_DEGREE_DEV;
    int *PEg = Dtg + SBP_MAX_DEGREE_DEV;
    const int tid = threadIdx.x;
    for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int g = find_graph(starts, nG, item);
        const GDev &d = G[g];
        const int v = d.hub[item - starts[g]];
        if (!in_batch(d, v)) continue;
        const int r = d.boff + d.lab[v];
        const int op = d.out_ptr[v], kout = d.out_ptr[v + 1] - op;
        const int ip = d.in_ptr[v], kin = d.in_ptr[v + 1] - ip;
        const int k = kout + kin;
        if (k > SBP_MAX_DEGREE_DEV) {  // beyond the scratch (validation rejects such graphs): no move
            if (tid == 0) nb[d.voff + v] = -1;
            continue;
        }
        const Words4 W = draw_words(d.seed, (uint32_t)v, d.sweep, 0u, 0u);
        const double lnu = log(draw_unit(W.w[3]));
        int s;
        {
            const long long eC = (long long)d.eps * d.C;
            const int j = (int)draw_idx(W.w[0], (uint64_t)k);
            const int u = j < kout ? d.out_idx[op + j] : d.in_idx[ip + (j - kout)];
            const int t = d.boff + d.lab[u];
            const long long dt = (long long)bm.dout[t] + bm.din[t];
            if (draw_idx(W.w[1], (uint64_t)(dt + eC)) < eC) s = d.boff + (int)draw_idx(W.w[2], (uint64_t)d.C);
            else s = s_draw_wave(bm, bm.rptr[t] + bm.cptr[t], bm.rptr[t + 1] + bm.cptr[t + 1], draw_idx(W.w[2], (uint64_t)dt));
        }
        if (s == r) {
            if (tid == 0) {
                MoveOut o;
                o.s = s;
                record_move(d, v, r, o, true, nb, tr);
            }
            continue;
        }
        int m = 2;
        while (m < k) m <<= 1;
        if (m <= HUB_LDS)
            hub_move(d, bm, v, r, s, op, kout, ip, kin, m, HUB_LDS, lnu, Ks, Dts, PEs, nb, tr, H);
        else
            hub_move(d, bm, v, r, s, op, kout, ip, kin, m, SBP_MAX_DEGREE_DEV, lnu, Kg, Dtg, PEg, nb, tr, H);
        __syncthreads();
    }
}

__global__ void k_sweep_apply(const GDev *__restrict__ G, const int *__restrict__ vstart, int nG, int Ntot,
                              const int *__restrict__ nb) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < Ntot; i += gridDim.x * blockDim.x) {
        const int g = find_graph(vstart, nG, i);
        const GDev &d = G[g];
        if (d.action != ACT_SWEEP && d.action != ACT_DSWEEP) continue;
        const int v = i - d.voff;
        if (!in_batch(d, v)) continue;
        const int x = nb[i];
        if (x >= 0) d.lab[v] = x;
    }
}

// ---------------------------------------------------------------- merge scoring
// -(change of L) when union blocks A and B become one block (Alg. 1).
__device__ double merge_dL(const SparseBM &bm, int A, int B) {
    const int lane = threadIdx.x & 63;
    double acc = 0.0;
    {
        const int la = bm.rptr[A + 1] - bm.rptr[A], lb = bm.rptr[B + 1] - bm.rptr[B];
        const int X = la <= lb ? A : B, Y = la <= lb ? B : A;
        const int x0 = bm.rptr[X], x1 = bm.rptr[X + 1];
        for (int q = x0 + lane; q < x1; q += 64) {
            const int t = bm.rcol[q];
            if (t == A || t == B) continue;
            const int y = m_get(bm, Y, t);
            if (y) {
                const int x = bm.rval[q];
                acc += xlogx((double)(x + y)) - xlogx((double)x) - xlogx((double)y);
            }
        }
    }
    {
        const int la = bm.cptr[A + 1] - bm.cptr[A], lb = bm.cptr[B + 1] - bm.cptr[B];
        const int X = la <= lb ? A : B, Y = la <= lb ? B : A;
        const int x0 = bm.cptr[X], x1 = bm.cptr[X + 1];
        for (int q = x0 + lane; q < x1; q += 64) {
            const int t = bm.crow[q];
            if (t == A || t == B) continue;
            const int y = mt_get(bm, Y, t);
            if (y) {
                const int x = bm.cval[q];
                acc += xlogx((double)(x + y)) - xlogx((double)x) - xlogx((double)y);
            }
        }
    }
    if (lane == 0) {
        const int a = m_get(bm, A, A), b = m_get(bm, A, B), e = m_get(bm, B, A), g = m_get(bm, B, B);
        acc += xlogx((double)(a + b + e + g)) - xlogx((double)a) - xlogx((double)b) - xlogx((double)e) -
               xlogx((double)g);
        const double oa = bm.dout[A], ob = bm.dout[B], ia = bm.din[A], ib = bm.din[B];
        acc -= xlogx(oa + ob) - xlogx(oa) - xlogx(ob);
        acc -= xlogx(ia + ib) - xlogx(ia) - xlogx(ib);
    }
    return wave_sum(acc);
}

// Divide-and-conquer combination (Alg. 3): for every community C1 + c2 the
// community c1 < C1 of the first result whose merge with it has the smallest
// floor(dS_local 2^20) (dS_local = -(change of L), as for Alg. 1), the lowest
// c1 on ties.  A wave per c2, the candidates c1 in ascending order.
__global__ void __launch_bounds__(BLK) k_combine_choice(SparseBM bm, int C1, int C2, int *__restrict__ best) {
    const int lane = threadIdx.x & 63;
    const int gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    for (int c2 = gw; c2 < C2; c2 += nw) {
        int b = -1;
        long long bk = INT64_MAX;
        for (int c1 = 0; c1 < C1; ++c1) {
            const long long key = merge_rank(-merge_dL(bm, C1 + c2, c1));
            if (b < 0 || key < bk) {
                b = c1;
                bk = key;
            }
        }
        if (lane == 0) best[c2] = b;
    }
}

// Row A and column A of M staged in LDS for the merge proposals of block A
// (at most MERGE_ROW entries each); lds_find reads the entry at index b of a
// staged list (0 where absent).
constexpr int MERGE_ROW = 256;
__device__ __forceinline__ int lds_find(const int *__restrict__ c, const int *__restrict__ v, int n, int b) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (c[mid] < b) lo = mid + 1; else hi = mid;
    }
    return (lo < n && c[lo] == b) ? v[lo] : 0;
}
// merge_dL with row A and column A of M staged in LDS (ac/av: columns and
// values of row A, la entries; rc/rv: rows and values of column A, lc
// entries), evaluated by an aligned group of 8 lanes (gl = lane in the group),
// each group with its own B: the group walks row B and column B in global
// memory and finds the matching entries of A in LDS.  The same terms as
// merge_dL; every lane of the group ends with the sum.
__device__ double merge_dL_grp8(const SparseBM &bm, int A, int B, const int *ac, const int *av, int la,
                                const int *rc, const int *rv, int lc, int gl) {
    double acc = 0.0;
    for (int q = bm.rptr[B] + gl; q < bm.rptr[B + 1]; q += 8) {
        const int t = bm.rcol[q];
        if (t == A || t == B) continue;
        const int x = lds_find(ac, av, la, t);
        if (x) {
            const int y = bm.rval[q];
            acc += xlogx((double)(x + y)) - xlogx((double)x) - xlogx((double)y);
        }
    }
    for (int q = bm.cptr[B] + gl; q < bm.cptr[B + 1]; q += 8) {
        const int t = bm.crow[q];
        if (t == A || t == B) continue;
        const int x = lds_find(rc, rv, lc, t);
        if (x) {
            const int y = bm.cval[q];
            acc += xlogx((double)(x + y)) - xlogx((double)x) - xlogx((double)y);
        }
    }
    if (gl == 0) {
        const int a = lds_find(ac, av, la, A), b = lds_find(ac, av, la, B), e = lds_find(rc, rv, lc, B);
        const int g = m_get(bm, B, B);
        acc += xlogx((double)(a + b + e + g)) - xlogx((double)a) - xlogx((double)b) - xlogx((double)e) -
               xlogx((double)g);
        const double oa = bm.dout[A], ob = bm.dout[B], ia = bm.din[A], ib = bm.din[B];
        acc -= xlogx(oa + ob) - xlogx(oa) - xlogx(ob);
        acc -= xlogx(ia + ib) - xlogx(ia) - xlogx(ib);
    }
    return grp8_sum(acc);
}

__global__ void __launch_bounds__(BLK) k_merge_scores(const GDev *__restrict__ G, const int *__restrict__ bstart, int nG,
                                                     int n_items, SparseBM bm, int *__restrict__ partner,
                                                     double *__restrict__ dS, double *__restrict__ dSl) {
    __shared__ int sAc[BLK / 64][MERGE_ROW], sAv[BLK / 64][MERGE_ROW], sRc[BLK / 64][MERGE_ROW], sRv[BLK / 64][MERGE_ROW];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    for (int item = gw; item < n_items; item += nw) {
        const int g = find_graph(bstart, nG, item);
        const GDev &d = G[g];
        const int c = item - bstart[g];
        const int A = d.boff + c;
        const int C = d.C;
        const long long dc = (long long)bm.dout[A] + bm.din[A];
        const long long eC = (long long)d.eps * C;
        int best = -1;
        double bestL = 0.0;
        long long bestkey = INT64_MAX;
        // row A and column A in LDS when short enough, for all the proposals
        const int ra = bm.rptr[A], la = bm.rptr[A + 1] - ra, ca = bm.cptr[A], lc = bm.cptr[A + 1] - ca;
        const bool staged = la <= MERGE_ROW && lc <= MERGE_ROW;
        if (staged) {
            for (int q = lane; q < la; q += 64) {
                sAc[wv][q] = bm.rcol[ra + q];
                sAv[wv][q] = bm.rval[ra + q];
            }
            for (int q = lane; q < lc; q += 64) {
                sRc[wv][q] = bm.crow[ca + q];
                sRv[wv][q] = bm.cval[ca + q];
            }
        }
        wave_sync_lds();
        // the partners of 64 proposals at a time: lane l draws proposal j0 + l
        for (int j0 = 0; j0 < d.proposals && C > 1; j0 += 64) {
        int cp_lane = c;
        if (j0 + lane < d.proposals) {
            const int j = j0 + lane;
            const Words4 W = draw_words(d.seed, (uint32_t)c, d.phase, (uint32_t)(2 * j), 1u);
            if (dc == 0) {
                const int kk = (int)draw_idx(W.w[2], (uint64_t)(C - 1));
                cp_lane = kk + (kk >= c);
            } else {
                const int t = s_draw(bm, A, draw_idx(W.w[0], (uint64_t)dc));
                const long long dt = (long long)bm.dout[t] + bm.din[t];
                if (draw_idx(W.w[1], (uint64_t)(dt + eC)) < eC) {
                    const int kk = (int)draw_idx(W.w[2], (uint64_t)(C - 1));
                    cp_lane = kk + (kk >= c);
                } else {
                    cp_lane = s_draw(bm, t, draw_idx(W.w[2], (uint64_t)dt)) - d.boff;
                }
            }
        }
        const int n_here = d.proposals - j0 < 64 ? d.proposals - j0 : 64;
        if (staged) {
            // eight proposals at a time, one per group of 8 lanes; then taken
            // in proposal order
            const int gl = lane & 7, grp = lane >> 3;
            for (int jb = 0; jb < n_here; jb += 8) {
                const int jj = jb + grp;
                const int cpg = __shfl(cp_lane, jj < n_here ? jj : 0, SBP_WAVE);
                const bool ok = jj < n_here && cpg != c;
                const double lg = -merge_dL_grp8(bm, A, d.boff + (ok ? cpg : c), sAc[wv], sAv[wv], la, sRc[wv],
                                                 sRv[wv], lc, gl);
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int cp = __shfl(cpg, 8 * q, SBP_WAVE);
                    const double local = __shfl(lg, 8 * q, SBP_WAVE);
                    if (jb + q >= n_here || cp == c) continue;
                    const long long key = merge_rank(local);
                    if (key < bestkey) {
                        bestkey = key;
                        best = cp;
                        bestL = local;
                    }
                }
            }
            continue;
        }
        for (int jj = 0; jj < n_here; ++jj) {
            const int cp = __shfl(cp_lane, jj, SBP_WAVE);
            if (cp == c) continue;
            const double local = -merge_dL(bm, A, d.boff + cp);
            const long long key = merge_rank(local);
            if (key < bestkey) {
                bestkey = key;
                best = cp;
                bestL = local;
            }
        }
        }
        if (lane == 0) {
            const double inf = __builtin_huge_val();
            partner[d.boff + c] = best;
            dSl[d.boff + c] = best < 0 ? inf : bestL;
            const double off = C > 1 ? model_terms((double)d.e, (double)d.n, (double)(C - 1)) -
                                           model_terms((double)d.e, (double)d.n, (double)C)
                                     : 0.0;
            dS[d.boff + c] = best < 0 ? inf : bestL + off;
        }
        wave_sync_lds();
    }
}

// ---------------------------------------------------------------- merge application
// Items are the blocks of the merging graphs, item i = bstart[g] + c.
__global__ void k_mkeys(const GDev *__restrict__ G, const int *__restrict__ bstart, int nG, int n_items,
                        const double *__restrict__ dSl, uint64_t *__restrict__ key, uint64_t *__restrict__ val) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_items; i += gridDim.x * blockDim.x) {
        const int g = find_graph(bstart, nG, i);
        const GDev &d = G[g];
        const long long r = merge_rank(dSl[d.boff + (i - bstart[g])]);
        key[i] = (uint64_t)r ^ 0x8000000000000000ull;
        val[i] = (uint64_t)i;
    }
}
__global__ void k_mgraph_keys(const int *__restrict__ bstart, int nG, int n_items, const uint64_t *__restrict__ val,
                              uint64_t *__restrict__ key) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n_items; q += gridDim.x * blockDim.x)
        key[q] = (uint64_t)find_graph(bstart, nG, (int)val[q]);
}
// pos[item] = rank within its graph; jump/max init for the cycle search
__global__ void k_minit(const GDev *__restrict__ G, const int *__restrict__ bstart, int nG, int n_items,
                        const uint64_t *__restrict__ sorted_items, const int *__restrict__ partner,
                        int *__restrict__ pos, int *__restrict__ jump, int *__restrict__ mx,
                        int *__restrict__ oncyc) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n_items; q += gridDim.x * blockDim.x) {
        const int i = (int)sorted_items[q];
        const int g = find_graph(bstart, nG, i);
        const GDev &d = G[g];
        int p = partner[d.boff + (i - bstart[g])];
        if (p >= d.C) p = -1;  // out-of-range partners count as none
        pos[i] = q - bstart[g];
        jump[i] = p >= 0 ? bstart[g] + p : i;
        mx[i] = p >= 0 ? q - bstart[g] : -1;
        oncyc[i] = 0;
    }
}
__global__ void k_mdouble(int n_items, const int *__restrict__ j0, const int *__restrict__ m0, int *__restrict__ j1,
                          int *__restrict__ m1) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_items; i += gridDim.x * blockDim.x) {
        const int a = j0[i];
        j1[i] = j0[a];
        if (m0) m1[i] = max(m0[i], m0[a]);
    }
}
__global__ void k_mmark(int n_items, const int *__restrict__ jump, int *__restrict__ oncyc) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_items; i += gridDim.x * blockDim.x) oncyc[jump[i]] = 1;
}
// flag in sorted order: valid partner and not the closing edge of a cycle
__global__ void k_mflags(const GDev *__restrict__ G, const int *__restrict__ bstart, int nG, int n_items,
                         const uint64_t *__restrict__ sorted_items, const int *__restrict__ partner,
                         const int *__restrict__ pos, const int *__restrict__ mx, const int *__restrict__ oncyc,
                         int *__restrict__ flag) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n_items; q += gridDim.x * blockDim.x) {
        const int i = (int)sorted_items[q];
        const int g = find_graph(bstart, nG, i);
        const GDev &d = G[g];
        const int p = partner[d.boff + (i - bstart[g])];
        const bool valid = p >= 0 && p < d.C;
        const bool closes = oncyc[i] && pos[i] == mx[i];
        flag[q] = (valid && !closes) ? 1 : 0;
    }
}
// accepted edges: the first `merges` flagged candidates of each graph
__global__ void k_maccept(const GDev *__restrict__ G, const int *__restrict__ bstart, int nG, int n_items,
                          const uint64_t *__restrict__ sorted_items, const int *__restrict__ partner,
                          const int *__restrict__ flag, const long long *__restrict__ ex, int *__restrict__ jump) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n_items; q += gridDim.x * blockDim.x) {
        const int i = (int)sorted_items[q];
        const int g = find_graph(bstart, nG, i);
        const GDev &d = G[g];
        const long long before = ex[q] - ex[bstart[g]];
        const bool acc = flag[q] && before < d.merges;
        jump[i] = acc ? bstart[g] + partner[d.boff + (i - bstart[g])] : i;
    }
}
__global__ void k_mlow_init(int n_items, int *__restrict__ low) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_items; i += gridDim.x * blockDim.x) low[i] = 0x7fffffff;
}
__global__ void k_mlow(int n_items, const int *__restrict__ root, int *__restrict__ low) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_items; i += gridDim.x * blockDim.x)
        atomicMin(&low[root[i]], i);
}
__global__ void k_mrep(int n_items, const int *__restrict__ root, const int *__restrict__ low, int *__restrict__ rep) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_items; i += gridDim.x * blockDim.x)
        rep[i] = (low[root[i]] == i) ? 1 : 0;
}
// map[item] = new local label; per-graph new block count
__global__ void k_mmap(const int *__restrict__ bstart, int nG, int n_items, const int *__restrict__ root,
                       const int *__restrict__ low, const long long *__restrict__ ex, int *__restrict__ map) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_items; i += gridDim.x * blockDim.x) {
        const int g = find_graph(bstart, nG, i);
        map[i] = (int)(ex[low[root[i]]] - ex[bstart[g]]);
    }
}
// per-graph count of flagged items (exclusive scan ex with total at ex[n_items])
__global__ void k_group_counts(const int *__restrict__ bstart, int nG, int n_items, const long long *__restrict__ ex,
                               int *__restrict__ gC) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nG) return;
    const int lo = bstart[g], hi = g + 1 < nG ? bstart[g + 1] : n_items;
    gC[g] = (int)(ex[hi] - ex[lo]);
}
// lab <- map[blkstart[g] + lab] over the vertex items
__global__ void k_relabel(const GDev *__restrict__ G, const int *__restrict__ vstart, int nG, int n_vitems,
                          const int *__restrict__ blkstart, const int *__restrict__ map) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_vitems; i += gridDim.x * blockDim.x) {
        const int g = find_graph(vstart, nG, i);
        const GDev &d = G[g];
        const int v = i - vstart[g];
        d.lab[v] = map[blkstart[g] + d.lab[v]];
    }
}
// compaction: occupied labels
__global__ void k_occupied(const GDev *__restrict__ G, const int *__restrict__ vstart, int nG, int n_vitems,
                           const int *__restrict__ blkstart, int *__restrict__ occ) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_vitems; i += gridDim.x * blockDim.x) {
        const int g = find_graph(vstart, nG, i);
        const GDev &d = G[g];
        occ[blkstart[g] + d.lab[i - vstart[g]]] = 1;
    }
}
__global__ void k_compact_map(const int *__restrict__ bstart, int nG, int n_items, const long long *__restrict__ ex,
                              int *__restrict__ map) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_items; i += gridDim.x * blockDim.x) {
        const int g = find_graph(bstart, nG, i);
        map[i] = (int)(ex[i] - ex[bstart[g]]);
    }
}

// ---------------------------------------------------------------- graph ingest
// key = a * n + b for edge (a, b); flags an endpoint outside [0, n)
__global__ void k_edge_pair_keys(const int *__restrict__ a, const int *__restrict__ b, long long e, int n,
                                 uint64_t *__restrict__ keys, int *__restrict__ flag) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < e; i += (long long)gridDim.x * blockDim.x) {
        const int x = a[i], y = b[i];
        if (x < 0 || x >= n || y < 0 || y >= n) {
            atomicOr(flag, 1);
            keys[i] = 0;
        } else {
            keys[i] = (uint64_t)x * (uint64_t)n + (uint64_t)y;
        }
    }
}
__global__ void k_split_keys(const uint64_t *__restrict__ keys, long long e, int n, int *__restrict__ hi,
                             int *__restrict__ lo) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < e; i += (long long)gridDim.x * blockDim.x) {
        hi[i] = (int)(keys[i] / (uint64_t)n);
        lo[i] = (int)(keys[i] % (uint64_t)n);
    }
}
__global__ void k_set_count(long long *p, long long v) { *p = v; }

}  // namespace

size_t hub_scratch_ints_per_slot() { return HUB_SLOT_INTS; }
int dl_chunks_of(int e, int C) { return (e + DL_CHUNK - 1) / DL_CHUNK + (2 * C + DL_CHUNK - 1) / DL_CHUNK; }

// ---------------------------------------------------------------- host launchers
int build_union_sparse(const GDev *dG, const StepMeta &m, SparseBM &bm, UnionScratch &ws, hipStream_t s) {
    const long long Etot = m.Etot;
    const int Ctot = m.Ctot;
    bm.Ctot = Ctot;
    int rc;
    // 1. one key per edge: (block of source) * Ctot + block of target, sorted
    hipLaunchKernelGGL(k_edge_keys, dim3(grid_for(m.Ntot, BLK, 16384)), dim3(BLK), 0, s, dG, m.voff, m.G, (int)m.Ntot,
                       Ctot, ws.k0);
    SBP_LAUNCH_CHECK();
    if ((rc = radix_sort(ws.k0, ws.k1, nullptr, nullptr, Etot, ceil_log2((uint64_t)Ctot * (uint64_t)Ctot), ws.temp, s)))
        return rc;
    // 2. run-length encode into the row lists
    int *flags = ws.i0, *urow = ws.i1, *start = bm.crow;  // crow is free until step 3
    hipLaunchKernelGGL(k_rle_flags, dim3(grid_for(Etot, BLK, 8192)), dim3(BLK), 0, s, ws.k0, Etot, flags);
    SBP_LAUNCH_CHECK();
    if ((rc = scan_exclusive_i32(flags, ws.s0, Etot, bm.nnz, ws.temp, s))) return rc;
    hipLaunchKernelGGL(k_rle_emit, dim3(grid_for(Etot, BLK, 8192)), dim3(BLK), 0, s, ws.k0, flags, ws.s0, Etot, Ctot,
                       urow, bm.rcol, start);
    hipLaunchKernelGGL(k_rle_count, dim3(grid_for(Etot, BLK, 8192)), dim3(BLK), 0, s, start, bm.nnz, Etot, bm.rval);
    hipLaunchKernelGGL(k_lower_bounds, dim3(grid_for(Ctot + 1, BLK, 8192)), dim3(BLK), 0, s, urow, bm.nnz, Ctot,
                       bm.rptr);
    SBP_LAUNCH_CHECK();
    // 3. columns: stable sort of the entries by column (padding sorts last)
    hipLaunchKernelGGL(k_csc_keys, dim3(grid_for(Etot, BLK, 8192)), dim3(BLK), 0, s, urow, bm.rcol, bm.rval, bm.nnz,
                       Etot, Ctot, ws.k0, ws.v0);
    SBP_LAUNCH_CHECK();
    if ((rc = radix_sort(ws.k0, ws.k1, ws.v0, ws.v1, Etot, ceil_log2((uint64_t)Ctot + 1), ws.temp, s))) return rc;
    int *ccol = ws.i0;
    hipLaunchKernelGGL(k_csc_emit, dim3(grid_for(Etot, BLK, 8192)), dim3(BLK), 0, s, ws.k0, ws.v0, bm.nnz, ccol,
                       bm.crow, bm.cval);
    hipLaunchKernelGGL(k_lower_bounds, dim3(grid_for(Ctot + 1, BLK, 8192)), dim3(BLK), 0, s, ccol, bm.nnz, Ctot,
                       bm.cptr);
    SBP_LAUNCH_CHECK();
    // 4. degrees and proposal tables, wave per block
    hipLaunchKernelGGL(k_block_rows, dim3(grid_for((long long)Ctot * 64, BLK, 8192)), dim3(BLK), 0, s, bm);
    SBP_LAUNCH_CHECK();
    return 0;
}

int union_dl(const GDev *dG, const StepMeta &m, const SparseBM &bm, UnionScratch &ws, hipStream_t s) {
    if (m.n_chunks > 0)
        hipLaunchKernelGGL(k_dl_partial, dim3(m.n_chunks), dim3(BLK), 0, s, dG, m.chstart, m.G, m.n_chunks, bm,
                           ws.dl_part);
    hipLaunchKernelGGL(k_dl_final, dim3(m.G), dim3(64), 0, s, dG, m.chstart, m.G, m.n_chunks, ws.dl_part,
                       ws.dl);
    SBP_LAUNCH_CHECK();
    return 0;
}

// A second stream per device for work that overlaps the caller's stream
// within one call, forked and joined with events; default priority.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    std::mutex mu;  // one fork-join sequence at a time
};
constexpr int SIDE_DEVICES = 64;
static SideStream g_side[SIDE_DEVICES];
static std::mutex g_side_init;

static int side_stream(SideStream **out) {
    int dev = 0;
    SBP_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= SIDE_DEVICES) return fail(-5, "device index beyond the side-stream table");
    std::lock_guard<std::mutex> lk(g_side_init);
    SideStream &S = g_side[dev];
    if (!S.s) {
        SBP_HIP_CHECK(hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking));
        SBP_HIP_CHECK(hipEventCreateWithFlags(&S.fork, hipEventDisableTiming));
        SBP_HIP_CHECK(hipEventCreateWithFlags(&S.join, hipEventDisableTiming));
    }
    *out = &S;
    return 0;
}

// Evaluation of one batch on two streams: hubs and the 9-32-end vertices on
// the side stream, the other vertices on the caller's.  All kernels read the
// same snapshot and write disjoint proposals; the caller's stream waits for
// the side stream before the labels are applied.
int union_sweep(const GDev *dG, const StepMeta &m, const SparseBM &bm, UnionScratch &ws, const SweepTraceDev &tr,
                hipStream_t s) {
    {
    ProfileScope prof("sweep_eval", s);
    int rc;
    SideStream *side = nullptr;
    if ((rc = side_stream(&side))) return rc;
    std::lock_guard<std::mutex> lk(side->mu);
    SBP_HIP_CHECK(hipEventRecord(side->fork, s));
    SBP_HIP_CHECK(hipStreamWaitEvent(side->s, side->fork, 0));
    if (m.n_hub > 0) {
        const int grid = m.n_hub < ws.hub_slots ? m.n_hub : ws.hub_slots;
        hipLaunchKernelGGL(k_sweep_hub, dim3(grid), dim3(HUB_THREADS), 0, side->s, dG, m.hub, m.G, m.n_hub, bm, ws.nb,
                           tr, ws.hub_scratch);
        SBP_LAUNCH_CHECK();
    }
    if (m.n_leaf > 0) {
        const long long tiles = ((long long)m.n_leaf + 63) / 64;
        hipLaunchKernelGGL(k_sweep_small<16>, dim3(grid_for(tiles, SMALL_WAVES, 16384)), dim3(SMALL_WAVES * 64), 0,
                           side->s, dG, m.leaf, m.G, m.n_leaf, bm, ws.nb, tr);
        hipLaunchKernelGGL(k_sweep_small<32>, dim3(grid_for(tiles, SMALL_WAVES, 16384)), dim3(SMALL_WAVES * 64), 0,
                           side->s, dG, m.leaf, m.G, m.n_leaf, bm, ws.nb, tr);
        hipLaunchKernelGGL(k_sweep_small<8>, dim3(grid_for(tiles, SMALL_WAVES, 16384)), dim3(SMALL_WAVES * 64), 0, s,
                           dG, m.leaf, m.G, m.n_leaf, bm, ws.nb, tr);
        hipLaunchKernelGGL(k_sweep_leaf, dim3(grid_for(tiles, LEAF_WAVES, 16384)), dim3(LEAF_WAVES * 64), 0, s, dG,
                           m.leaf, m.G, m.n_leaf, bm, ws.nb, tr);
        SBP_LAUNCH_CHECK();
    }
    SBP_HIP_CHECK(hipEventRecord(side->join, side->s));
    SBP_HIP_CHECK(hipStreamWaitEvent(s, side->join, 0));
    }
    hipLaunchKernelGGL(k_sweep_apply, dim3(grid_for(m.Ntot, BLK, 8192)), dim3(BLK), 0, s, dG, m.voff, m.G,
                       (int)m.Ntot, ws.nb);
    SBP_LAUNCH_CHECK();
    return 0;
}

// The graph owning union block t (blocks of graph g are [boff, boff + C)).
__device__ __forceinline__ int graph_of_block(const GDev *G, int nG, int t) {
    int lo = 0, hi = nG - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (G[mid].boff <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Lookup tables of M (C x C ints, graph-local ids) of the graphs that have
// one: a wave per union block zeroes its table row, then (second launch, so
// every zero lands first) a wave per union block writes its sparse row.
// Blocks past a graph's (lowered) count have no row.
__global__ void __launch_bounds__(BLK) k_table_zero_rows(const GDev *__restrict__ G, int nG, int Ctot) {
    const int lane = threadIdx.x & 63;
    const int gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    for (int t = gw; t < Ctot; t += nw) {
        const GDev &d = G[graph_of_block(G, nG, t)];
        const int a = t - d.boff;
        if (!d.mdense || a >= d.C) continue;
        int *__restrict__ row = d.mdense + (size_t)a * d.C;
        for (int x = lane; x < d.C; x += 64) row[x] = 0;
    }
}
__global__ void __launch_bounds__(BLK) k_table_fill_rows(const GDev *__restrict__ G, int nG, int Ctot, SparseBM bm) {
    const int lane = threadIdx.x & 63;
    const int gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    for (int t = gw; t < Ctot; t += nw) {
        const GDev &d = G[graph_of_block(G, nG, t)];
        const int a = t - d.boff;
        if (!d.mdense || a >= d.C) continue;
        int *__restrict__ row = d.mdense + (size_t)a * d.C;
        for (int q = bm.rptr[t] + lane; q < bm.rptr[t + 1]; q += 64) row[bm.rcol[q] - d.boff] = bm.rval[q];
    }
}

// ---------------------------------------------------------------- build from tables
// When every graph of a step has a C x C table (C <= SBP_TABLE_MAX_C), M is
// counted straight into the tables (one integer atomic per edge), and the
// sorted rows, sorted columns, proposal rows with running sums and block
// degrees are read off the tables in ascending order: the same arrays as the
// sort-based build, at O(sum C^2) instead of several radix passes over the
// edges.

// M of every graph into its table (zeroed beforehand); edges in flattened
// per-block ranges as in k_edge_keys.
__global__ void __launch_bounds__(BLK) k_tab_hist(const GDev *__restrict__ G, const int *__restrict__ vstart, int nG,
                                                  int Ntot) {
    constexpr int HCELLS = SBP_DENSE_MAX_C_DEV * SBP_DENSE_MAX_C_DEV;
    __shared__ long long U[BLK + 1];
    __shared__ int gi[BLK], ra[BLK];
    __shared__ int H[HCELLS];  // a workgroup's own counts when its range lies in one graph with C <= 64
    for (int b0 = blockIdx.x * BLK; b0 < Ntot; b0 += gridDim.x * BLK) {
        const int nv = min(BLK, Ntot - b0);
        __syncthreads();
        if ((int)threadIdx.x < nv) {
            const int t = threadIdx.x, i = b0 + t;
            const int g = find_graph(vstart, nG, i);
            const GDev &d = G[g];
            const int v = i - d.voff;
            U[t] = d.eoff + d.out_ptr[v];
            ra[t] = d.lab[v] * d.C;
            gi[t] = g;
            if (t == nv - 1) U[nv] = d.eoff + d.out_ptr[v + 1];
        }
        __syncthreads();
        // one graph with few blocks: count in LDS first (many edges share a
        // handful of cells, which global atomics would serialise)
        const GDev &d0 = G[gi[0]];
        const bool local = gi[0] == gi[nv - 1] && d0.C <= SBP_DENSE_MAX_C_DEV;
        const int CC = local ? d0.C * d0.C : 0;
        for (int c = threadIdx.x; c < CC; c += BLK) H[c] = 0;
        __syncthreads();
        const long long e1 = U[nv];
        for (long long x = U[0] + threadIdx.x; x < e1; x += BLK) {
            int lo = 0, hi = nv - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (U[mid] <= x) lo = mid; else hi = mid - 1;
            }
            const GDev &d = G[gi[lo]];
            const int cell = ra[lo] + d.lab[d.out_idx[x - d.eoff]];
            if (local) atomicAdd(&H[cell], 1);
            else atomicAdd(&d.mdense[cell], 1);
        }
        __syncthreads();
        for (int c = threadIdx.x; c < CC; c += BLK)
            if (H[c]) atomicAdd(&d0.mdense[c], H[c]);
    }
}

// Per union block: nonzeros of its row and of its column, and the degrees.
__global__ void __launch_bounds__(BLK) k_tab_counts(const GDev *__restrict__ G, int nG, int Ctot, SparseBM bm,
                                                    int *__restrict__ rlen, int *__restrict__ clen) {
    const int lane = threadIdx.x & 63;
    const int gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    for (int t = gw; t < Ctot; t += nw) {
        const GDev &d = G[graph_of_block(G, nG, t)];
        const int a = t - d.boff;
        const int C = a < d.C ? d.C : 0;  // a block past the graph's (lowered) count is empty
        const int *__restrict__ T = d.mdense;
        int nr = 0, nc = 0, so = 0, si = 0;
        for (int x = lane; x < C; x += 64) {
            const int r = T[a * C + x], c = T[x * C + a];
            nr += r != 0;
            nc += c != 0;
            so += r;
            si += c;
        }
        nr = wave_sum_i32(nr);
        nc = wave_sum_i32(nc);
        so = wave_sum_i32(so);
        si = wave_sum_i32(si);
        if (lane == 0) {
            rlen[t] = nr;
            clen[t] = nc;
            bm.dout[t] = so;
            bm.din[t] = si;
        }
    }
}

__global__ void k_tab_ptrs(const long long *__restrict__ pr, const long long *__restrict__ pc,
                           const long long *__restrict__ tot, int Ctot, int *__restrict__ rptr, int *__restrict__ cptr,
                           long long *__restrict__ nnz) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t <= Ctot; t += gridDim.x * blockDim.x) {
        rptr[t] = t < Ctot ? (int)pr[t] : (int)tot[0];
        cptr[t] = t < Ctot ? (int)pc[t] : (int)tot[1];
        if (t == 0) *nnz = tot[0];
    }
}

// Rows, columns and proposal rows of every union block, in ascending order:
// a wave per block walks its table row and column 64 entries at a time and
// places the nonzeros by ballot.  The proposal row takes, per column s, the
// row entry (M_ts) then the column entry (M_st), with inclusive running sums.
__global__ void __launch_bounds__(BLK) k_tab_emit(const GDev *__restrict__ G, int nG, int Ctot, SparseBM bm) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = lanemask_lt();
    const int gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    for (int t = gw; t < Ctot; t += nw) {
        const GDev &d = G[graph_of_block(G, nG, t)];
        const int a = t - d.boff, b = d.boff;
        const int C = a < d.C ? d.C : 0;  // a block past the graph's (lowered) count is empty
        const int *__restrict__ T = d.mdense;
        int pr = bm.rptr[t], pc = bm.cptr[t], ps = bm.rptr[t] + bm.cptr[t];
        int carry = 0;
        for (int x0 = 0; x0 < C; x0 += 64) {
            const int x = x0 + lane;
            const int r = x < C ? T[a * C + x] : 0, c = x < C ? T[x * C + a] : 0;
            const uint64_t mr = __ballot(r != 0), mc = __ballot(c != 0);
            if (r) {
                const int k = pr + __popcll(mr & below);
                bm.rcol[k] = b + x;
                bm.rval[k] = r;
            }
            if (c) {
                const int k = pc + __popcll(mc & below);
                bm.crow[k] = b + x;
                bm.cval[k] = c;
            }
            // proposal row: lane x holds up to two entries, row entry first
            const int n_here = (r != 0) + (c != 0);
            int off = n_here, v = r + c;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {  // inclusive scans of entry counts and values
                const int y = __shfl_up(off, o, SBP_WAVE), z = __shfl_up(v, o, SBP_WAVE);
                if (lane >= o) {
                    off += y;
                    v += z;
                }
            }
            const int k0 = ps + off - n_here;  // the lane's first slot
            const int base = carry + v - (r + c);
            if (r) {
                bm.scol[k0] = b + x;
                bm.scum[k0] = base + r;
            }
            if (c) {
                bm.scol[k0 + (r != 0)] = b + x;
                bm.scum[k0 + (r != 0)] = base + r + c;
            }
            pr += __popcll(mr);
            pc += __popcll(mc);
            ps += __shfl(off, 63, SBP_WAVE);
            carry += __shfl(v, 63, SBP_WAVE);
        }
    }
}

int build_union_from_tables(const GDev *dG, const StepMeta &m, SparseBM &bm, UnionScratch &ws,
                            const int *list, int n_list, hipStream_t s) {
    const int Ctot = m.Ctot;
    bm.Ctot = Ctot;
    (void)list;
    (void)n_list;
    hipLaunchKernelGGL(k_table_zero_rows, dim3(grid_for((long long)Ctot * 64, BLK, 8192)), dim3(BLK), 0, s, dG, m.G,
                       Ctot);
    hipLaunchKernelGGL(k_tab_hist, dim3(grid_for(m.Ntot, BLK, 16384)), dim3(BLK), 0, s, dG, m.voff, m.G,
                       (int)m.Ntot);
    int *rlen = ws.i0, *clen = ws.i1;
    hipLaunchKernelGGL(k_tab_counts, dim3(grid_for((long long)Ctot * 64, BLK, 8192)), dim3(BLK), 0, s, dG, m.G, Ctot,
                       bm, rlen, clen);
    SBP_LAUNCH_CHECK();
    int rc;
    long long *tot = (long long *)ws.v1;  // two totals (the sort buffers are not used on this path)
    if ((rc = scan_exclusive_i32(rlen, ws.s0, Ctot, tot + 0, ws.temp, s))) return rc;
    if ((rc = scan_exclusive_i32(clen, ws.s1, Ctot, tot + 1, ws.temp, s))) return rc;
    hipLaunchKernelGGL(k_tab_ptrs, dim3(grid_for(Ctot + 1, BLK, 4096)), dim3(BLK), 0, s, (const long long *)ws.s0,
                       (const long long *)ws.s1, (const long long *)tot, Ctot, bm.rptr, bm.cptr, bm.nnz);
    hipLaunchKernelGGL(k_tab_emit, dim3(grid_for((long long)Ctot * 64, BLK, 8192)), dim3(BLK), 0, s, dG, m.G, Ctot, bm);
    SBP_LAUNCH_CHECK();
    return 0;
}

int union_lookup_tables(const GDev *dG, int nG, int n_list, const SparseBM &bm, hipStream_t s) {
    if (n_list <= 0) return 0;
    const int grid = grid_for((long long)bm.Ctot * 64, BLK, 8192);
    hipLaunchKernelGGL(k_table_zero_rows, dim3(grid), dim3(BLK), 0, s, dG, nG, bm.Ctot);
    hipLaunchKernelGGL(k_table_fill_rows, dim3(grid), dim3(BLK), 0, s, dG, nG, bm.Ctot, bm);
    SBP_LAUNCH_CHECK();
    return 0;
}

int union_combine_choice(const SparseBM &bm, int C1, int C2, int *best, hipStream_t s) {
    if (C2 <= 0) return 0;
    hipLaunchKernelGGL(k_combine_choice, dim3(grid_for((long long)C2 * 64, BLK, 16384)), dim3(BLK), 0, s, bm, C1, C2,
                       best);
    SBP_LAUNCH_CHECK();
    return 0;
}

int union_merge_scores(const GDev *dG, const StepMeta &m, const SparseBM &bm, int *partner, double *dS, double *dSl,
                       hipStream_t s) {
    if (m.n_mblk <= 0) return 0;
    hipLaunchKernelGGL(k_merge_scores, dim3(grid_for((long long)m.n_mblk * 64, BLK, 16384)), dim3(BLK), 0, s, dG,
                       m.mblk, m.G, m.n_mblk, bm, partner, dS, dSl);
    SBP_LAUNCH_CHECK();
    return 0;
}

int union_merge_apply(const GDev *dG, const StepMeta &m, const int *partner, const double *dSl, UnionScratch &ws,
                      hipStream_t s) {
    const int n = m.n_mblk;
    if (n <= 0) return 0;
    const int grid = grid_for(n, BLK, 8192);
    const int G = m.G;
    const int *bstart = m.mblk;
    int rc;
    // order by (rank of dS_local, block): sort by rank, then stably by graph
    hipLaunchKernelGGL(k_mkeys, dim3(grid), dim3(BLK), 0, s, dG, bstart, G, n, dSl, ws.k0, ws.v0);
    SBP_LAUNCH_CHECK();
    if ((rc = radix_sort(ws.k0, ws.k1, ws.v0, ws.v1, n, 64, ws.temp, s))) return rc;
    if (G > 1) {
        hipLaunchKernelGGL(k_mgraph_keys, dim3(grid), dim3(BLK), 0, s, bstart, G, n, ws.v0, ws.k0);
        SBP_LAUNCH_CHECK();
        if ((rc = radix_sort(ws.k0, ws.k1, ws.v0, ws.v1, n, ceil_log2((uint64_t)G), ws.temp, s))) return rc;
    }
    const uint64_t *sorted = ws.v0;
    int *j0 = ws.mj0, *j1 = ws.mj1, *m0 = ws.mm0, *m1 = ws.mm1;
    hipLaunchKernelGGL(k_minit, dim3(grid), dim3(BLK), 0, s, dG, bstart, G, n, sorted, partner, ws.mpos, j0, m0,
                       ws.mcyc);
    SBP_LAUNCH_CHECK();
    // the closing edge of each proposal cycle: largest rank on the cycle
    const int rounds = ceil_log2((uint64_t)(m.maxC_merge > 1 ? m.maxC_merge : 2)) + 1;
    for (int it = 0; it < rounds; ++it) {
        hipLaunchKernelGGL(k_mdouble, dim3(grid), dim3(BLK), 0, s, n, j0, m0, j1, m1);
        int *t = j0; j0 = j1; j1 = t;
        t = m0; m0 = m1; m1 = t;
    }
    hipLaunchKernelGGL(k_mmark, dim3(grid), dim3(BLK), 0, s, n, j0, ws.mcyc);
    int *flag = ws.i0;
    hipLaunchKernelGGL(k_mflags, dim3(grid), dim3(BLK), 0, s, dG, bstart, G, n, sorted, partner, ws.mpos, m0, ws.mcyc,
                       flag);
    SBP_LAUNCH_CHECK();
    if ((rc = scan_exclusive_i32(flag, ws.s0, n, nullptr, ws.temp, s))) return rc;
    // joins: the first `merges` remaining candidates; groups by pointer jumping
    hipLaunchKernelGGL(k_maccept, dim3(grid), dim3(BLK), 0, s, dG, bstart, G, n, sorted, partner, flag, ws.s0, j0);
    for (int it = 0; it < rounds; ++it) {
        hipLaunchKernelGGL(k_mdouble, dim3(grid), dim3(BLK), 0, s, n, j0, (const int *)nullptr, j1, (int *)nullptr);
        int *t = j0; j0 = j1; j1 = t;
    }
    const int *root = j0;
    hipLaunchKernelGGL(k_mlow_init, dim3(grid), dim3(BLK), 0, s, n, ws.mlow);
    hipLaunchKernelGGL(k_mlow, dim3(grid), dim3(BLK), 0, s, n, root, ws.mlow);
    hipLaunchKernelGGL(k_mrep, dim3(grid), dim3(BLK), 0, s, n, root, ws.mlow, ws.i1);
    SBP_LAUNCH_CHECK();
    if ((rc = scan_exclusive_i32(ws.i1, ws.s1, n, ws.s1 + n, ws.temp, s))) return rc;
    hipLaunchKernelGGL(k_mmap, dim3(grid), dim3(BLK), 0, s, bstart, G, n, root, ws.mlow, ws.s1, ws.mmap);
    hipLaunchKernelGGL(k_group_counts, dim3((G + 63) / 64), dim3(64), 0, s, bstart, G, n, ws.s1, ws.gC);
    SBP_LAUNCH_CHECK();
    return 0;
}

int union_compact(const GDev *dG, const StepMeta &m, UnionScratch &ws, hipStream_t s) {
    const int n = m.n_cblk;
    if (n <= 0) return 0;
    int rc;
    if ((rc = fill_i32(ws.i0, 0, n, s))) return rc;
    if (m.n_cvtx > 0) {
        hipLaunchKernelGGL(k_occupied, dim3(grid_for(m.n_cvtx, BLK, 8192)), dim3(BLK), 0, s, dG, m.cvtx, m.G, m.n_cvtx,
                           m.cblk, ws.i0);
        SBP_LAUNCH_CHECK();
    }
    if ((rc = scan_exclusive_i32(ws.i0, ws.s1, n, ws.s1 + n, ws.temp, s))) return rc;
    hipLaunchKernelGGL(k_compact_map, dim3(grid_for(n, BLK, 8192)), dim3(BLK), 0, s, m.cblk, m.G, n, ws.s1, ws.mmap);
    hipLaunchKernelGGL(k_group_counts, dim3((m.G + 63) / 64), dim3(64), 0, s, m.cblk, m.G, n, ws.s1, ws.gC);
    SBP_LAUNCH_CHECK();
    return 0;
}

// CSR (sorted by source, then target) and CSC (by target, then source) of an
// edge list; flag (device) is set to 1 if an endpoint lies outside [0, n).
int graph_from_edges(int n, long long e, const int *src, const int *dst, int *out_ptr, int *out_idx, int *in_ptr,
                     int *in_idx, UnionScratch &ws, long long *count, int *flag, hipStream_t s) {
    const int grid = grid_for(e, BLK, 8192);
    const int bits = ceil_log2((uint64_t)n * (uint64_t)n);
    int rc;
    hipLaunchKernelGGL(k_set_count, dim3(1), dim3(1), 0, s, count, e);
    for (int pass = 0; pass < 2; ++pass) {
        const int *a = pass == 0 ? src : dst, *b = pass == 0 ? dst : src;
        int *ptr = pass == 0 ? out_ptr : in_ptr, *idx = pass == 0 ? out_idx : in_idx;
        if (e > 0) {
            hipLaunchKernelGGL(k_edge_pair_keys, dim3(grid), dim3(BLK), 0, s, a, b, e, n, ws.k0, flag);
            SBP_LAUNCH_CHECK();
            if ((rc = radix_sort(ws.k0, ws.k1, nullptr, nullptr, e, bits, ws.temp, s))) return rc;
            hipLaunchKernelGGL(k_split_keys, dim3(grid), dim3(BLK), 0, s, ws.k0, e, n, ws.i0, idx);
        }
        hipLaunchKernelGGL(k_lower_bounds, dim3(grid_for(n + 1, BLK, 8192)), dim3(BLK), 0, s, ws.i0, count, n, ptr);
        SBP_LAUNCH_CHECK();
    }
    return 0;
}

int union_relabel(const GDev *dG, int G, const int *vstart, int n_vitems, const int *blkstart, const int *map,
                  hipStream_t s) {
    if (n_vitems <= 0) return 0;
    hipLaunchKernelGGL(k_relabel, dim3(grid_for(n_vitems, BLK, 8192)), dim3(BLK), 0, s, dG, vstart, G, n_vitems,
                       blkstart, map);
    SBP_LAUNCH_CHECK();
    return 0;
}

}  // namespace sbp
