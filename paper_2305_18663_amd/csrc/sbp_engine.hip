// sbp_engine.hip -- C-ABI entry points and the batched partition engine.
//
// Every public call runs the batched kernels on a batch of one graph, so a
// graph's result does not depend on whether it ran alone or in a batch.
//
// Engine step (one host synchronisation per step):
//   1. upload the layout (union offsets from the block counts known on the
//      host, which may be upper bounds right after a merge or compaction);
//   2. fix the block counts on the device from the authoritative copy;
//   3. rebuild the union blockmodel and the DL of every graph;
//   4. read the DLs and block counts back and synchronise;
//   5. advance every graph's own partition (Sec. II-B): MCMC stop test
//      (Alg. 2), golden-ratio search over C, next merge target (Alg. 1);
//   6. launch this step's actions against the blockmodel of 3: one sweep
//      batch, a merge phase (scoring + application), a compaction, or a
//      copy of a stored assignment into the working one.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/sbp.h"
#include "sbp_internal.h"

namespace sbp {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

// ---------------------------------------------------------------- kernel timing
static std::mutex g_prof_mu;
static int g_prof_stride = 0;  // 0: off; k: events on every k-th launch of each named kernel
struct ProfRec {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    long long calls = 0;  // launches since profiling was enabled
};
static std::map<std::string, ProfRec> g_prof;

ProfileScope::ProfileScope(const char *name, hipStream_t stream, bool attach) : s(stream), attach_(attach) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (g_prof_stride <= 0) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;  // no timing events inside a captured graph
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    if (g_prof[name].calls++ % g_prof_stride != 0) return;  // not a sampled launch
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
    }
    ProfRec &r = g_prof[name];
    r.ev.push_back({a, b});
    slot = (int)r.ev.size() - 1;
    name_ = name;
    if (attach_) {
        start = a;
        stop = b;
    } else {
        (void)hipEventRecord(a, s);
    }
}
ProfileScope::~ProfileScope() {
    if (slot < 0 || attach_) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    (void)hipEventRecord(g_prof[name_].ev[slot].second, s);
}

static std::mutex g_trace_mu;
static std::map<long long, std::pair<std::vector<long long>, std::vector<double>>> g_traces;

namespace {

constexpr int BLK = 256;

inline size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

// ---------------------------------------------------------------- small kernels
__global__ void k_validate(const int *__restrict__ ptr, const int *__restrict__ idx, const int *__restrict__ optr,
                           int n, int e, int *__restrict__ flags) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += gridDim.x * blockDim.x) {
        if (v == 0 && ptr[0] != 0) atomicOr(flags, 1);
        if (v == n) {
            if (ptr[n] != e) atomicOr(flags, 1);
            continue;
        }
        const int a = ptr[v], b = ptr[v + 1];
        if (b < a || a < 0 || b > e) {
            atomicOr(flags, 1);
            continue;
        }
        const int deg = (b - a) + (optr[v + 1] - optr[v]);
        if (deg > SBP_MAX_DEGREE_DEV) atomicOr(flags, 2);
        for (int j = a; j < b; ++j)
            if (idx[j] < 0 || idx[j] >= n) {
                atomicOr(flags, 1);
                break;
            }
    }
}
__global__ void k_check_labels(const int *__restrict__ lab, int n, int C, int *__restrict__ flag) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        if (lab[v] < 0 || lab[v] >= C) atomicOr(flag, 1);
}
__global__ void k_fix_C(GDev *__restrict__ G, int nG, const int *__restrict__ Cdev) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < nG) G[g].C = Cdev[G[g].slot];
}
__global__ void k_store_C(const GDev *__restrict__ G, int nG, int act, const int *__restrict__ gC, int *__restrict__ Cdev) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < nG && G[g].action == act) Cdev[G[g].slot] = gC[g];
}
__global__ void k_set_i32(int *p, int v) { *p = v; }
__global__ void k_zero_stats(sbp_sweep_stats_dev *st) {
    st->proposals = st->self_proposals = st->accepted = st->near_ties = 0;
    st->sum_dS_accepted = 0.0;
    st->dl_after = 0.0;
}
// hub list of a graph (order irrelevant: each vertex's move depends only on its own data)
__global__ void k_hub_list(const int *__restrict__ optr, const int *__restrict__ iptr, int n, int *__restrict__ hub,
                           int *__restrict__ count) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        if ((optr[v + 1] - optr[v]) + (iptr[v + 1] - iptr[v]) > SBP_LEAF_MAX) hub[atomicAdd(count, 1)] = v;
}
// sweep totals from the per-vertex status: per-workgroup partials over a fixed
// split of the batch's vertices, then one workgroup adds them in order
__global__ void __launch_bounds__(256) k_sweep_stats_part(const signed char *__restrict__ status,
                                                         const double *__restrict__ dS, int n, int batch,
                                                         int n_batches, const int *__restrict__ skip,
                                                         long long *__restrict__ part,
                                                         double *__restrict__ sum_part) {
    __shared__ long long a[4], b[4], c[4], e[4];
    __shared__ double d[4];
    long long np = 0, ns = 0, na = 0, nt = 0;
    double sd = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x;; i += (long long)gridDim.x * 256) {
        const long long v = batch + n_batches * i;
        if (v >= n) break;
        if (skip && skip[v] > 0) continue;  // a hub, moved before the batches
        ++np;
        const int x = status[v];  // -1 no-op, else accepted (bit 0) and near tie (bit 1)
        if (x < 0) ++ns;
        if (x >= 0 && (x & 1)) {
            ++na;
            sd += dS[v];
        }
        if (x >= 0 && (x & 2)) ++nt;
    }
    np = wave_sum_i64(np);
    ns = wave_sum_i64(ns);
    na = wave_sum_i64(na);
    nt = wave_sum_i64(nt);
    sd = wave_sum(sd);
    if ((threadIdx.x & 63) == 0) {
        a[threadIdx.x >> 6] = np;
        b[threadIdx.x >> 6] = ns;
        c[threadIdx.x >> 6] = na;
        e[threadIdx.x >> 6] = nt;
        d[threadIdx.x >> 6] = sd;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long p = 0, q = 0, r = 0, u = 0;
        double t = 0.0;
        for (int w = 0; w < 4; ++w) {
            p += a[w];
            q += b[w];
            r += c[w];
            u += e[w];
            t += d[w];
        }
        part[4 * blockIdx.x + 0] = p;
        part[4 * blockIdx.x + 1] = q;
        part[4 * blockIdx.x + 2] = r;
        part[4 * blockIdx.x + 3] = u;
        sum_part[blockIdx.x] = t;
    }
}
__global__ void __launch_bounds__(64) k_sweep_stats_final(const long long *__restrict__ part,
                                                          const double *__restrict__ sum_part, int nblk,
                                                          const double *__restrict__ dl,
                                                          sbp_sweep_stats_dev *__restrict__ st) {
    const int lane = threadIdx.x;
    long long p = 0, q = 0, r = 0, u = 0;
    double t = 0.0;
    for (int w = lane; w < nblk; w += 64) {
        p += part[4 * w + 0];
        q += part[4 * w + 1];
        r += part[4 * w + 2];
        u += part[4 * w + 3];
        t += sum_part[w];
    }
    p = wave_sum_i64(p);
    q = wave_sum_i64(q);
    r = wave_sum_i64(r);
    u = wave_sum_i64(u);
    t = wave_sum(t);
    if (lane == 0) {
        st->proposals += p;
        st->self_proposals += q;
        st->accepted += r;
        st->near_ties += u;
        st->sum_dS_accepted += t;
        if (dl) st->dl_after = *dl;
    }
}
__global__ void k_copy_dl(const double *__restrict__ src, double *__restrict__ dst) { *dst = *src; }
__global__ void k_relabel_map(int *__restrict__ lab, const int *__restrict__ map, int n) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) lab[v] = map[lab[v]];
}
__global__ void k_iota(int *__restrict__ p, int n) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) p[v] = v;
}
__global__ void k_dense_coo(const int *__restrict__ M, const int *__restrict__ dout, const int *__restrict__ din, int C,
                            int *__restrict__ rows, int *__restrict__ cols, int *__restrict__ vals,
                            int *__restrict__ odout, int *__restrict__ odin, long long *__restrict__ nnz) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    long long k = 0;
    for (int a = 0; a < C; ++a)
        for (int b = 0; b < C; ++b) {
            const int x = M[a * C + b];
            if (x) {
                rows[k] = a;
                cols[k] = b;
                vals[k] = x;
                ++k;
            }
        }
    for (int a = 0; a < C; ++a) {
        odout[a] = dout[a];
        odin[a] = din[a];
    }
    *nnz = k;
}
__global__ void k_sparse_rows(const int *__restrict__ rptr, int C, int *__restrict__ rows) {
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < C; a += gridDim.x * blockDim.x)
        for (int k = rptr[a]; k < rptr[a + 1]; ++k) rows[k] = a;
}

// ---------------------------------------------------------------- layouts
struct BMView {
    bool dense;
    DenseBM d;
    int *delta;
    SparseBM sp;
    double *dl;
    long long *spare;  // one word for small readbacks
    size_t bytes;
};

BMView bm_layout(void *base, int n, int e, int C) {
    (void)n;
    const long long e_al = ((long long)(e > 0 ? e : 1) + 255) & ~255ll;
    Arena a(base, SIZE_MAX);
    if (!base) a = Arena::measure();
    BMView v{};
    v.dense = C <= SBP_DENSE_MAX_C;
    if (v.dense) {
        v.d.C = C;
        v.d.M = a.take<int>((size_t)C * C);
        v.d.fM = a.take<double>((size_t)C * C);
        v.d.dout = a.take<int>(C);
        v.d.din = a.take<int>(C);
        v.d.dl = a.take<double>(1);
        v.delta = a.take<int>((size_t)C * C);
        v.d.ftab_max = (unsigned)(e > 0 ? e : 0);
        v.d.ftab = a.take<double>((size_t)v.d.ftab_max + 1);
        v.d.nl = a.take<unsigned char>(2 * (size_t)e_al);
        v.d.nl_in = e_al;
        v.d.bounds = a.take<int>(SBP_DENSE_BOUNDS);
        v.d.mir_o = a.take<int>((size_t)e_al);
        v.d.mir_i = a.take<int>((size_t)e_al);
        v.d.flags = a.take<int>(4);
        v.dl = v.d.dl;
        v.spare = a.take<long long>(1);
    } else {
        const long long cap = e > 0 ? e : 1;
        v.sp.Ctot = C;
        v.sp.cap = cap;
        v.sp.rptr = a.take<int>((size_t)C + 1);
        v.sp.rcol = a.take<int>(cap);
        v.sp.rval = a.take<int>(cap);
        v.sp.cptr = a.take<int>((size_t)C + 1);
        v.sp.crow = a.take<int>(cap);
        v.sp.cval = a.take<int>(cap);
        v.sp.scol = a.take<int>(2 * cap);
        v.sp.scum = a.take<int>(2 * cap);
        v.sp.dout = a.take<int>(C);
        v.sp.din = a.take<int>(C);
        v.sp.nnz = a.take<long long>(1);
        v.dl = a.take<double>(1);
        v.spare = a.take<long long>(1);
    }
    v.bytes = a.used;
    return v;
}

int hub_slots_for(long long e) {
    long long h = 2 * e / (SBP_LEAF_MAX + 1) + 1;
    if (h > 256) h = 256;
    return (int)h;
}

// Union scratch for capacities (vertices, edges, graphs).
struct UnionLayout {
    SparseBM bm;
    UnionScratch ws;
    GDev *dG;
    int *meta;        // 8 G starts
    int *Cdev;        // [G] authoritative block counts
    int *partner;     // [N]
    double *dS, *dSl; // [N]
    int *hub_count;   // device counter for on-the-fly hub lists
    int *flags;       // validation flags
    double *ftab;     // f(x) = x ln x for 0 <= x <= max(E, 1): no count of any graph exceeds it
    unsigned ftab_max;
    char *dslots;     // per engine slot: dense M, f(M) and degrees for C <= 64
    void *dmulti;     // launch tables of the multi-graph dense sweep
    int *tables;      // C x C lookup tables of M for the sparse sweeps of a step
    long long table_ints;
    int *tlist;       // [G] graphs given a table this step
    size_t bytes;
};

// One engine slot's dense blockmodel: M [64*64] ints, f(M) [64*64] doubles,
// degrees [64] + [64] ints (rows packed at the graph's own C).
constexpr size_t DSLOT_BYTES = 64 * 64 * 4 + 64 * 64 * 8 + 2 * 64 * 4;
int g_engine_dense_max_c = SBP_DENSE_MAX_C;  // engine sweeps at C <= this use the dense kernels (0: never)
int g_table_max_c = SBP_TABLE_MAX_C;         // sparse sweeps at C <= this read M from a lookup table (0: never)
int g_table_ratio = 4;  // automatic table builds need ratio * cost <= 16 * edges (4: cost <= 4 E)
int g_table_build = 1;  // count M into the tables: 0 never, 1 when they are small against the edges, 2 whenever all fit
int g_batches_in_step = 1;  // a sweep's later hubs and batches run in the step of its first (0: one a step)

UnionLayout union_layout(Arena &a, long long N, long long E, int G) {
    UnionLayout u{};
    const long long cap = std::max<long long>(std::max(N, E), 1);
    u.bm.cap = cap;
    u.bm.rptr = a.take<int>(N + 1);
    u.bm.rcol = a.take<int>(cap);
    u.bm.rval = a.take<int>(cap);
    u.bm.cptr = a.take<int>(N + 1);
    u.bm.crow = a.take<int>(cap);
    u.bm.cval = a.take<int>(cap);
    u.bm.scol = a.take<int>(2 * cap);
    u.bm.scum = a.take<int>(2 * cap);
    u.bm.dout = a.take<int>(N + 1);
    u.bm.din = a.take<int>(N + 1);
    u.bm.nnz = a.take<long long>(1);
    UnionScratch &w = u.ws;
    w.k0 = a.take<uint64_t>(cap);
    w.k1 = a.take<uint64_t>(cap);
    w.v0 = a.take<uint64_t>(cap);
    w.v1 = a.take<uint64_t>(cap);
    w.s0 = a.take<long long>(cap + 1);
    w.s1 = a.take<long long>(cap + 1);
    w.i0 = a.take<int>(cap);
    w.i1 = a.take<int>(cap);
    w.temp = a.take<char>(std::max(radix_temp_bytes(cap), scan_temp_bytes(cap)));
    const long long chunks = (E + 2 * N) / 2048 + 2 * (long long)G + 2;
    w.dl_part = a.take<double>(chunks);
    w.dl = a.take<double>(G);
    w.nb = a.take<int>(N);
    w.hub_slots = hub_slots_for(E);
    w.hub_scratch = a.take<int>((size_t)w.hub_slots * hub_scratch_ints_per_slot());
    w.mpos = a.take<int>(N);
    w.mj0 = a.take<int>(N);
    w.mj1 = a.take<int>(N);
    w.mm0 = a.take<int>(N);
    w.mm1 = a.take<int>(N);
    w.mcyc = a.take<int>(N);
    w.mlow = a.take<int>(N);
    w.mmap = a.take<int>(N);
    w.gC = a.take<int>(G);
    u.dG = a.take<GDev>(G);
    u.meta = a.take<int>(8 * (size_t)G + 8);
    u.Cdev = a.take<int>(G);
    u.partner = a.take<int>(N);
    u.dS = a.take<double>(N);
    u.dSl = a.take<double>(N);
    u.hub_count = a.take<int>(1);
    u.flags = a.take<int>(4);
    u.ftab_max = (unsigned)std::max<long long>(E, 1);
    u.ftab = a.take<double>((size_t)u.ftab_max + 1);
    u.dslots = a.take<char>(DSLOT_BYTES * (size_t)G);
    u.dmulti = a.take<char>(dense_multi_scratch_bytes(G));
    {
        // tables for block counts up to SBP_TABLE_MAX_C, at most 256 MB
        const long long cmax = std::min<long long>(N, SBP_TABLE_MAX_C);
        long long t = std::min<long long>(64LL << 20, cmax * cmax * std::max(1, std::min(G, 64)));
        t = std::min(t, std::max<long long>(N, 1) * SBP_TABLE_MAX_C);
        u.table_ints = std::max<long long>(t, 1);
    }
    u.tables = a.take<int>((size_t)u.table_ints);
    u.tlist = a.take<int>(G);
    u.bytes = a.used;
    return u;
}

// Host image of the step metadata; `dev` resolves the start arrays.
struct HostMeta {
    std::vector<int> buf;  // 8 arrays of G
    StepMeta m{};
    void init(int G) {
        buf.assign(8 * (size_t)G, 0);
        m = StepMeta{};
        m.G = G;
    }
    int *arr(int k) { return buf.data() + (size_t)k * m.G; }
    void bind(int *dev) {
        const int G = m.G;
        m.voff = dev;
        m.chstart = dev + G;
        m.leaf = dev + 2 * G;
        m.hub = dev + 3 * G;
        m.mblk = dev + 4 * G;
        m.mvtx = dev + 5 * G;
        m.cblk = dev + 6 * G;
        m.cvtx = dev + 7 * G;
    }
};

// Fill layout and work lists from the host descriptors (with actions set).
void plan_step(std::vector<GDev> &hG, HostMeta &hm) {
    const int G = (int)hG.size();
    hm.init(G);
    long long N = 0, E = 0;
    int Ctot = 0, ch = 0, nl = 0, nh = 0, mb = 0, mv = 0, cb = 0, cv = 0, maxC = 1;
    for (int g = 0; g < G; ++g) {
        GDev &d = hG[g];
        d.voff = (int)N;
        d.boff = Ctot;
        d.eoff = E;
        hm.arr(0)[g] = (int)N;
        hm.arr(1)[g] = ch;
        hm.arr(2)[g] = nl;
        hm.arr(3)[g] = nh;
        hm.arr(4)[g] = mb;
        hm.arr(5)[g] = mv;
        hm.arr(6)[g] = cb;
        hm.arr(7)[g] = cv;
        N += d.n;
        E += d.e;
        Ctot += d.C;
        ch += dl_chunks_of(d.e, d.C);
        if (d.action == ACT_SWEEP) {
            nl += d.n;
            nh += d.n_hub;
        } else if (d.action == ACT_MERGE) {
            mb += d.C;
            mv += d.n;
            maxC = std::max(maxC, d.C);
        } else if (d.action == ACT_COMPACT) {
            cb += d.C;
            cv += d.n;
        }
    }
    StepMeta &m = hm.m;
    m.n_chunks = ch;
    m.n_leaf = nl;
    m.n_hub = nh;
    m.n_mblk = mb;
    m.n_mvtx = mv;
    m.n_cblk = cb;
    m.n_cvtx = cv;
    m.Ctot = Ctot;
    m.maxC_merge = maxC;
    m.Ntot = N;
    m.Etot = E;
}

int upload_step(std::vector<GDev> &hG, HostMeta &hm, UnionLayout &u, hipStream_t s) {
    SBP_HIP_CHECK(hipMemcpyAsync(u.dG, hG.data(), hG.size() * sizeof(GDev), hipMemcpyHostToDevice, s));
    SBP_HIP_CHECK(hipMemcpyAsync(u.meta, hm.buf.data(), hm.buf.size() * sizeof(int), hipMemcpyHostToDevice, s));
    hm.bind(u.meta);
    return 0;
}

GDev gdev_of(const sbp_graph *g, int *lab, int C) {
    GDev d{};
    d.out_ptr = g->out_ptr;
    d.out_idx = g->out_idx;
    d.in_ptr = g->in_ptr;
    d.in_idx = g->in_idx;
    d.lab = lab;
    d.n = g->n;
    d.e = g->e;
    d.C = C;
    d.n_batches = 1;
    d.eps = 1;
    d.beta = 1.0;
    return d;
}

int check_graph_args(const sbp_graph *g) {
    if (!g) return fail(SBP_E_ARG, "null graph");
    if (g->n < 1 || g->e < 0) return fail(SBP_E_ARG, "graph needs n >= 1 and e >= 0");
    if (g->n >= (1 << 30) || g->e >= (1 << 30)) return fail(SBP_E_LIMIT, "n and e must be below 2^30");
    if (!g->out_ptr || !g->in_ptr || (g->e > 0 && (!g->out_idx || !g->in_idx)))
        return fail(SBP_E_ARG, "null graph array");
    return 0;
}

// Workspace of the single-graph calls: union scratch for one graph + lists.
struct SingleWS {
    UnionLayout u;
    int *hub;          // [n]
    signed char *status;
    double *dS;
    int *nb_dense;     // [n]
    long long *stats_part;
    double *sum_part;
    sbp_sweep_stats_dev *stats;
    size_t bytes;
};

SingleWS single_layout(void *base, size_t cap, int n, int e) {
    Arena a = base ? Arena(base, cap) : Arena::measure();
    SingleWS w{};
    w.u = union_layout(a, n, e, 1);
    w.hub = a.take<int>(n);
    w.status = a.take<signed char>(n);
    w.dS = a.take<double>(n);
    w.nb_dense = a.take<int>(n);
    const int nwg = dense_workgroups();
    w.stats_part = a.take<long long>(4 * ((size_t)nwg + 1));  // + the hybrid sweep's sequential pass
    w.sum_part = a.take<double>((size_t)nwg + 1);
    w.stats = a.take<sbp_sweep_stats_dev>(1);
    w.bytes = a.used;
    return w;
}

int check_sweep_args(const sbp_graph *g, const int32_t *assign, int32_t C, const void *bm,
                     const sbp_sweep_params *p) {
    int rc;
    if ((rc = check_graph_args(g))) return rc;
    if (!assign || !bm || !p || C < 1 || C > g->n || p->n_batches < 1 || p->eps < 0 || !(p->beta > 0))
        return fail(SBP_E_ARG, "bad sweep arguments");
    if (p->n_hubs < 0 || p->n_hubs > std::min(g->n, SBP_HUBS_MAX))
        return fail(SBP_E_ARG, "n_hubs must lie in [0, min(n, 4096)]");
    return 0;
}

SweepTraceDev trace_of(const sbp_sweep_trace *trace) {
    SweepTraceDev tr{};
    if (trace) {
        tr.prop = trace->prop;
        tr.dS = trace->dS;
        tr.lnH = trace->lnH;
        tr.margin = trace->margin;
        tr.accept = trace->accept;
    }
    return tr;
}

GDev sweep_desc(const sbp_graph *g, int32_t *assign, int32_t C, const sbp_sweep_params *p) {
    GDev d = gdev_of(g, assign, C);
    d.seed = p->seed;
    d.sweep = p->sweep;
    d.beta = p->beta;
    d.eps = p->eps;
    d.n_batches = std::min(p->n_batches, g->n);
    d.action = ACT_SWEEP;
    return d;
}

// One sweep on the dense tier: the optional sequential hub pass, then the
// batches (the first batch starts the totals in st).
int dense_sweep(GDev d, BMView &bv, DenseScratch &ds, int n_hubs, const HubScratch &hs, const SweepTraceDev &tr,
                sbp_sweep_stats_dev *st, hipStream_t s) {
    int rc;
    ds.delta = bv.delta;
    if ((rc = dense_hub_pass(d, bv.d, ds, n_hubs, hs, tr, s))) return rc;
    for (int b = 0; b < d.n_batches; ++b) {
        d.batch = b;
        if ((rc = dense_sweep_batch(d, bv.d, ds, tr, st, s))) return rc;
        ds.hub_slot = -1;  // the first batch folded the sequential pass into the totals
    }
    if (d.n_batches > 1) return dense_refresh_ends(d, bv.d, s);
    return 0;
}

// The dense tier's scratch inside a single-graph workspace.
void dense_scratch_of(const SingleWS &w, DenseScratch &ds, HubScratch &hs) {
    ds.nwg = dense_workgroups();
    ds.nb = w.nb_dense;
    ds.stats_part = w.stats_part;
    ds.sum_part = w.sum_part;
    // hybrid schedule: the hubs one at a time, then the batches without them
    hs.k0 = w.u.ws.k0;
    hs.k1 = w.u.ws.k1;
    hs.temp = w.u.ws.temp;
    hs.order = w.u.ws.i0;        // [cap >= n]
    hs.kk = w.u.ws.i1;           // [cap >= n]
    hs.hoff = (int *)w.u.ws.s0;  // [2 (cap + 1) >= n + 1]
    hs.codes = (int *)w.u.ws.v0; // [2 cap >= 2e]
    hs.mpos = (int *)w.u.ws.v1;  // [2 cap >= 2e]
    hs.hubrank = w.hub;          // [n]
}

}  // namespace

size_t sparse_one_bytes(int n, int e) { return single_layout(nullptr, 0, n, e).bytes; }

int build_sparse_one(const GDev &d0, void *ws, size_t ws_bytes, SparseBM &out, hipStream_t s) {
    SingleWS w = single_layout(ws, ws_bytes, d0.n, d0.e);
    if (!ws || ws_bytes < w.bytes) return fail(SBP_E_SPACE, "workspace too small");
    std::vector<GDev> hG{d0};
    hG[0].action = ACT_NONE;
    HostMeta hm;
    plan_step(hG, hm);
    int rc;
    if ((rc = upload_step(hG, hm, w.u, s))) return rc;
    out = w.u.bm;
    out.Ctot = d0.C;
    return build_union_sparse(w.u.dG, hm.m, out, w.u.ws, s);
}

namespace {

// ---------------------------------------------------------------- allocation-free sweep
// Scratch of sbp_nodal_sweep_static, a file-scope device array: the decision
// of every vertex (an int each, SBP_STATIC_MAX_VERTICES of them), the
// evaluation's per-workgroup partials (STATIC_MAX_WGS + 1 slots) and one
// statistics record for callers that pass none.  Every GPU the library runs
// on holds its own copy until the process ends; calls on one GPU share it.
// Nothing in it needs to start at zero: a sweep writes every decision and
// partial it later reads.
constexpr int STATIC_MAX_WGS = 4096;
constexpr size_t STATIC_NB_BYTES = (size_t)SBP_STATIC_MAX_VERTICES * 4;
constexpr size_t STATIC_PART_BYTES = (size_t)(STATIC_MAX_WGS + 1) * 4 * 8;
constexpr size_t STATIC_SUM_BYTES = (size_t)(STATIC_MAX_WGS + 1) * 8;
constexpr size_t STATIC_SCRATCH_BYTES = STATIC_NB_BYTES + STATIC_PART_BYTES + STATIC_SUM_BYTES + 256;
__device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

struct StaticScratch {
    int *nb;
    long long *stats_part;
    double *sum_part;
    sbp_sweep_stats_dev *stats;
};

std::mutex g_static_mu;
std::map<int, char *> g_static_ptr;  // device id -> address of that device's copy of scratch

// The current device's copy of scratch, looked up once per device (the
// array's name in host code is not a device address).
int static_scratch(StaticScratch &sc) {
    int dev = 0;
    SBP_HIP_CHECK(hipGetDevice(&dev));
    char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        auto it = g_static_ptr.find(dev);
        if (it == g_static_ptr.end()) {
            void *ptr = nullptr;
            SBP_HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            if (!ptr) return fail(SBP_E_HIP, "no device address for the static scratch array");
            it = g_static_ptr.emplace(dev, (char *)ptr).first;
        }
        base = it->second;
    }
    sc.nb = (int *)base;
    sc.stats_part = (long long *)(base + STATIC_NB_BYTES);
    sc.sum_part = (double *)(base + STATIC_NB_BYTES + STATIC_PART_BYTES);
    sc.stats = (sbp_sweep_stats_dev *)(base + STATIC_NB_BYTES + STATIC_PART_BYTES + STATIC_SUM_BYTES);
    return 0;
}

int build_one(const GDev &d0, UnionLayout &u, BMView &bv, hipStream_t s) {
    std::vector<GDev> hG{d0};
    hG[0].action = ACT_NONE;
    HostMeta hm;
    plan_step(hG, hm);
    int rc;
    if ((rc = upload_step(hG, hm, u, s))) return rc;
    SparseBM bm = bv.sp;
    bm.Ctot = d0.C;
    if ((rc = build_union_sparse(u.dG, hm.m, bm, u.ws, s))) return rc;
    if ((rc = union_dl(u.dG, hm.m, bm, u.ws, s))) return rc;
    hipLaunchKernelGGL(k_copy_dl, dim3(1), dim3(1), 0, s, (const double *)u.ws.dl, bv.dl);
    SBP_LAUNCH_CHECK();
    return 0;
}

}  // namespace

// ====================================================================== engine
struct GraphRun {
    long long tag = 0;
    sbp_graph g{};
    sbp_partition_params p{};
    int *lab = nullptr;  // working assignment (the caller's output array)
    int *slot_lab[3] = {nullptr, nullptr, nullptr};  // hi, mid, lo
    bool used[3] = {false, false, false};
    int slotC[3] = {0, 0, 0};
    double slotDL[3] = {0, 0, 0};
    int *hub = nullptr;
    int n_hub = 0;
    // hybrid sweeps (R21): the nh highest-degree vertices, in the order they
    // move; hub_rank[v] = position + 1 for them, 0 otherwise (device)
    int nh = 0;
    std::vector<int> hub_order;
    int *hub_rank = nullptr;
    int hub_i = -1;  // the hub of this step, or -1 during the batches
    size_t pool_off = 0, pool_bytes = 0;
    int eslot = 0;  // engine slot (index into Cdev)
    int C = 0;
    enum Phase { START, LOAD, PRE_MERGE, MERGED, MCMC, FINAL, DONE } phase = START;
    int action = ACT_NONE;
    int merges = 0;
    int C0 = 0, target = 0, C1 = 0, sweeps = 0, iters = 0, batch = 0;
    double tol = 0, dl_prev = 0;
    unsigned sweep_ctr = 0, phase_ctr = 0;
    int load_from = -1;
    std::vector<long long> trace;
    std::vector<double> trace_dl;
    double final_dl = 0;
    int final_C = 0;
};

struct sbp_engine_impl {
    hipStream_t s = nullptr;
    char *base = nullptr;
    size_t bytes = 0;
    long long maxV = 0, maxE = 0;
    int maxG = 0;
    size_t pool_bytes = 0;
    UnionLayout u{};
    std::vector<GraphRun *> active;
    std::vector<GraphRun *> finished;
    std::vector<std::pair<size_t, size_t>> free_list;  // (offset, bytes) of the pool
    std::vector<int> free_slots;
    long long usedV = 0, usedE = 0;
    std::vector<double> h_dl;
    std::vector<int> h_C;
};

}  // namespace sbp

struct sbp_engine : public sbp::sbp_engine_impl {};
struct sbp_sweep_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
    int dev;
};

namespace sbp {
namespace {

// Per-graph pool region: the three golden-search assignments, the hybrid
// sweep's hub ranks [n] and the list of vertices above SBP_LEAF_MAX ends.
size_t graph_bytes(int n, int e) {
    const long long hubs = 2LL * e / (SBP_LEAF_MAX + 1) + 2;
    return 4 * al((size_t)n * 4) + al((size_t)hubs * 4);
}

size_t pool_bound(long long V, long long E, int G) {
    return 16 * (size_t)V + 4 * (size_t)(2 * E / (SBP_LEAF_MAX + 1)) + (size_t)G * (5 * 256 + 64);
}

bool pool_alloc(sbp_engine *eng, size_t bytes, size_t &off) {
    for (size_t i = 0; i < eng->free_list.size(); ++i) {
        auto &f = eng->free_list[i];
        if (f.second >= bytes) {
            off = f.first;
            f.first += bytes;
            f.second -= bytes;
            if (f.second == 0) eng->free_list.erase(eng->free_list.begin() + i);
            return true;
        }
    }
    return false;
}

void pool_free(sbp_engine *eng, size_t off, size_t bytes) {
    eng->free_list.push_back({off, bytes});
    std::sort(eng->free_list.begin(), eng->free_list.end());
    std::vector<std::pair<size_t, size_t>> merged;
    for (auto &f : eng->free_list) {
        if (!merged.empty() && merged.back().first + merged.back().second == f.first) merged.back().second += f.second;
        else merged.push_back(f);
    }
    eng->free_list.swap(merged);
}

// golden-ratio search over C (Sec. II-B): insert a result
void golden_insert(GraphRun &r, int C, double dl, hipStream_t s) {
    // slots: 0 = hi, 1 = mid, 2 = lo
    auto set = [&](int k) {
        r.used[k] = true;
        r.slotC[k] = C;
        r.slotDL[k] = dl;
        (void)hipMemcpyAsync(r.slot_lab[k], r.lab, (size_t)r.g.n * 4, hipMemcpyDeviceToDevice, s);
    };
    auto swap = [&](int a, int b) {
        std::swap(r.used[a], r.used[b]);
        std::swap(r.slotC[a], r.slotC[b]);
        std::swap(r.slotDL[a], r.slotDL[b]);
        std::swap(r.slot_lab[a], r.slot_lab[b]);
    };
    if (!r.used[1]) {
        set(1);
    } else if (dl < r.slotDL[1]) {
        swap(C < r.slotC[1] ? 0 : 2, 1);
        set(1);
    } else {
        set(C < r.slotC[1] ? 2 : 0);
    }
}

// next (start slot, target) or -1 when the search is over
int golden_next(GraphRun &r, int &target) {
    if (r.iters >= r.p.max_iters) return -1;
    const bool hi = r.used[0], lo = r.used[2];
    const int Chi = r.slotC[0], Cmid = r.slotC[1], Clo = r.slotC[2];
    if (!lo) {
        const int merges = (int)std::floor(Cmid * r.p.merge_rate);
        if (merges < 1) return -1;
        target = Cmid - merges;
        return 1;
    }
    const int upper = hi ? Chi - Cmid : 0, lower = Cmid - Clo;
    if (hi ? (Chi - Clo <= 2) : (lower <= 1)) return -1;
    if (hi && upper >= lower) {
        int step = (int)std::floor(0.381966 * upper + 0.5);
        if (step < 1) step = 1;
        target = std::min(Cmid + step, Chi - 1);
        return 0;
    }
    int step = (int)std::floor(0.618034 * lower + 0.5);
    if (step < 1) step = 1;
    target = std::min(Clo + step, Cmid - 1);
    return 1;
}

// The search is over: the best stored assignment is loaded and compacted on
// the next step; the step after that reads its non-empty count and DL.
void start_final(sbp_engine *eng, GraphRun &r) {
    r.phase = GraphRun::FINAL;
    r.C = r.slotC[1];
    r.action = ACT_COMPACT;
    (void)hipMemcpyAsync(r.lab, r.slot_lab[1], (size_t)r.g.n * 4, hipMemcpyDeviceToDevice, eng->s);
}

// Trace row of the finished iteration and the result into the golden triple.
void store_result(sbp_engine *eng, GraphRun &r, double dl) {
    r.trace.insert(r.trace.end(), {(long long)r.C0, (long long)r.target, (long long)r.C1, (long long)r.sweeps,
                                   (long long)r.C1});
    r.trace_dl.push_back(dl);
    ++r.iters;
    golden_insert(r, r.C1, dl, eng->s);
}

// Advance one graph after its DL and block count were read back.
void advance(sbp_engine *eng, GraphRun &r, double dl, int C) {
    r.C = C;
    r.action = ACT_NONE;
    auto plan_next = [&]() {
        int target = 0;
        const int from = golden_next(r, target);
        if (from < 0) {
            start_final(eng, r);
            return;
        }
        r.C0 = r.slotC[from];
        r.target = target;
        r.load_from = from;
        // copy the stored assignment, rebuild on the next step, then merge
        (void)hipMemcpyAsync(r.lab, r.slot_lab[from], (size_t)r.g.n * 4, hipMemcpyDeviceToDevice, eng->s);
        r.C = r.C0;
        r.phase = GraphRun::PRE_MERGE;
    };
    switch (r.phase) {
    case GraphRun::START:
        golden_insert(r, C, dl, eng->s);
        plan_next();
        break;
    case GraphRun::PRE_MERGE:
        r.tol = r.used[2] ? r.p.t_post : r.p.t_pre;
        r.merges = r.C0 - r.target;
        r.action = ACT_MERGE;
        r.phase = GraphRun::MERGED;
        break;
    case GraphRun::MERGED:
        r.C1 = C;
        r.dl_prev = dl;
        r.sweeps = 0;
        r.batch = 0;
        if (r.p.max_sweeps < 1) {
            store_result(eng, r, dl);
            plan_next();
        } else {
            r.hub_i = r.nh > 0 ? 0 : -1;  // a hybrid sweep starts with its hubs
            r.action = ACT_SWEEP;
            r.phase = GraphRun::MCMC;
        }
        break;
    case GraphRun::MCMC: {
        const int nb = std::max(1, std::min(r.p.n_batches, r.g.n));
        if (r.hub_i >= 0) {  // the next hub, else the first batch
            if (++r.hub_i >= r.nh) {
                r.hub_i = -1;
                r.batch = 0;
            }
            r.action = ACT_SWEEP;
            break;
        }
        if (r.batch + 1 < nb) {
            ++r.batch;
            r.action = ACT_SWEEP;
            break;
        }
        ++r.sweeps;
        ++r.sweep_ctr;
        const bool stop = std::fabs(r.dl_prev - dl) < r.tol * dl || r.sweeps >= r.p.max_sweeps;
        r.dl_prev = dl;
        if (stop) {
            // the result is stored at the merged count: blocks the MCMC phase
            // emptied stay as empty labels
            store_result(eng, r, dl);
            plan_next();
        } else {
            r.batch = 0;
            r.hub_i = r.nh > 0 ? 0 : -1;
            r.action = ACT_SWEEP;
        }
        break;
    }
    case GraphRun::FINAL:
        r.phase = GraphRun::DONE;
        r.final_C = C;
        r.final_dl = dl;
        break;
    default:
        break;
    }
}

GDev desc_of(const GraphRun &r) {
    GDev d = gdev_of(&r.g, r.lab, r.C);
    d.hub = r.hub;
    d.n_hub = r.n_hub;
    d.slot = r.eslot;
    d.seed = r.p.seed;
    d.beta = r.p.beta;
    d.eps = r.p.eps;
    d.n_batches = std::max(1, std::min(r.p.n_batches, r.g.n));
    d.batch = r.batch;
    if (r.hub_i >= 0) {  // a hub alone: the batch {v : v mod n = hub}
        d.n_batches = r.g.n;
        d.batch = r.hub_order[r.hub_i];
    } else if (r.nh > 0) {
        d.skip = r.hub_rank;  // the batches skip the hubs
    }
    d.sweep = r.sweep_ctr;
    d.phase = r.phase_ctr;
    d.proposals = r.p.merge_proposals;
    d.merges = r.merges;
    d.action = r.action;
    return d;
}

// Layout, lookup tables and union blockmodel of the given graphs for one
// round of actions (descriptors without actions); with_dl: their DLs too.
struct StepState {
    std::vector<GDev> hG;
    HostMeta hm;
    std::vector<int *> tab;
    SparseBM bm;
};
int step_build(sbp_engine *eng, const std::vector<GraphRun *> &runs, StepState &st, bool with_dl) {
    hipStream_t s = eng->s;
    UnionLayout &u = eng->u;
    const int G = (int)runs.size();
    int rc;
    std::vector<GDev> &hG = st.hG;
    hG.assign(G, GDev{});
    // lookup tables of M for the graphs whose count (an upper bound: a merge
    // of the last step may have lowered it on the device) allows one, while
    // the space lasts; tables change no result, only the lookups' cost
    st.tab.assign(G, nullptr);
    std::vector<int> tlist;
    long long tused = 0;
    bool all_tabled = g_table_build > 0;  // every graph gets a table: M is counted into them
    {
        // worth it when the tables are small against the edges: the build
        // then scans sum C^2 entries (columns with a stride of C) instead of
        // radix-sorting every edge's key several times
        // (graphs above 64 blocks count with global atomics: at most 64 edges
        // per cell on average, or the atomics serialise)
        // cost model: a table scan against the sort of every edge key; columns
        // are read with a stride of C, which costs about four times more once
        // a table row no longer fits a few cache lines
        long long need = 0, cost = 0, edges = 0;
        bool spread = true;
        for (int g = 0; g < G && all_tabled; ++g) {
            const long long Cb = runs[g]->C, e = runs[g]->g.e;
            all_tabled = Cb <= g_table_max_c;
            need += (Cb * Cb + 63) & ~63LL;
            cost += Cb * Cb * (Cb > 512 ? 4 : 1);
            edges += e;
            spread = spread && (Cb <= SBP_DENSE_MAX_C || e <= 64 * Cb * Cb);
        }
        const bool cheap = spread && cost * g_table_ratio <= 16 * edges;
        all_tabled = all_tabled && need <= u.table_ints && (g_table_build == 2 || cheap);
    }
    for (int g = 0; g < G; ++g) {
        hG[g] = desc_of(*runs[g]);
        hG[g].action = ACT_NONE;
        const long long Cb = hG[g].C;
        if (all_tabled ||
            (Cb <= g_table_max_c && Cb > g_engine_dense_max_c && Cb * Cb <= u.table_ints - tused)) {
            st.tab[g] = u.tables + tused;
            tused += (Cb * Cb + 63) & ~63LL;
            hG[g].mdense = st.tab[g];
            tlist.push_back(g);
        }
    }
    plan_step(hG, st.hm);
    if ((rc = upload_step(hG, st.hm, u, s))) return rc;
    if (!tlist.empty())
        SBP_HIP_CHECK(hipMemcpyAsync(u.tlist, tlist.data(), tlist.size() * sizeof(int), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_fix_C, dim3((G + 63) / 64), dim3(64), 0, s, u.dG, G, (const int *)u.Cdev);
    SBP_LAUNCH_CHECK();
    st.bm = u.bm;
    if (all_tabled) {
        if ((rc = build_union_from_tables(u.dG, st.hm.m, st.bm, u.ws, u.tlist, G, s))) return rc;
    } else {
        if ((rc = build_union_sparse(u.dG, st.hm.m, st.bm, u.ws, s))) return rc;
        if ((rc = union_lookup_tables(u.dG, G, (int)tlist.size(), st.bm, s))) return rc;
    }
    if (with_dl && (rc = union_dl(u.dG, st.hm.m, st.bm, u.ws, s))) return rc;
    return 0;
}

// The actions the given graphs hold (GraphRun::action) against the blockmodel
// step_build made for the same list.
int step_act(sbp_engine *eng, const std::vector<GraphRun *> &runs, StepState &st) {
    hipStream_t s = eng->s;
    UnionLayout &u = eng->u;
    const int G = (int)runs.size();
    int rc;
    std::vector<GDev> &hG = st.hG;
    const HostMeta &hm = st.hm;
    SparseBM &bm = st.bm;
    bool any_act = false;
    std::vector<DenseSweepJob> djobs;
    for (int g = 0; g < G; ++g) {
        GraphRun &r = *runs[g];
        GDev d = desc_of(r);
        d.voff = hG[g].voff;
        d.boff = hG[g].boff;
        d.eoff = hG[g].eoff;
        d.C = r.C;
        if (r.action == ACT_MERGE) d.C = r.C0;
        d.mdense = st.tab[g];  // filled for the count the build used, which the actions keep
        if (r.action == ACT_SWEEP && d.C <= g_engine_dense_max_c) {
            // the dense kernels evaluate it; the union kernels apply it
            d.action = ACT_DSWEEP;
            char *slot = u.dslots + DSLOT_BYTES * (size_t)r.eslot;
            DenseSweepJob j;
            j.g = d;
            j.M = (int *)slot;
            j.fM = (double *)(slot + 64 * 64 * 4);
            j.dout = (int *)(slot + 64 * 64 * 12);
            j.din = j.dout + 64;
            j.nb = u.ws.nb + d.voff;
            djobs.push_back(j);
        }
        hG[g] = d;
        any_act |= r.action != ACT_NONE;
    }
    if (!any_act) return 0;
    // work lists for this round's actions (layout offsets kept from the build)
    HostMeta am;
    std::vector<GDev> tmp = hG;
    plan_step(tmp, am);
    for (int g = 0; g < G; ++g) am.arr(0)[g] = st.hm.arr(0)[g], am.arr(1)[g] = st.hm.arr(1)[g];
    am.m.Ctot = hm.m.Ctot;
    am.m.n_chunks = hm.m.n_chunks;
    if ((rc = upload_step(hG, am, u, s))) return rc;
    SweepTraceDev tr{};
    if (!djobs.empty() &&
        (rc = dense_multi_sweep(djobs, bm, u.ftab, u.ftab_max, u.dmulti, eng->maxG, s)))
        return rc;
    if (am.m.n_leaf + am.m.n_hub > 0 || !djobs.empty()) {
        StepMeta sm = am.m;
        sm.leaf = am.m.leaf;
        if ((rc = union_sweep(u.dG, sm, bm, u.ws, tr, s))) return rc;
    }
    if (am.m.n_mblk > 0) {
        if ((rc = union_merge_scores(u.dG, am.m, bm, u.partner, u.dS, u.dSl, s))) return rc;
        if ((rc = union_merge_apply(u.dG, am.m, u.partner, u.dSl, u.ws, s))) return rc;
        if ((rc = union_relabel(u.dG, G, am.m.mvtx, am.m.n_mvtx, am.m.mblk, u.ws.mmap, s))) return rc;
        hipLaunchKernelGGL(k_store_C, dim3((G + 63) / 64), dim3(64), 0, s, (const GDev *)u.dG, G, (int)ACT_MERGE,
                           (const int *)u.ws.gC, u.Cdev);
        SBP_LAUNCH_CHECK();
    }
    if (am.m.n_cblk > 0) {
        if ((rc = union_compact(u.dG, am.m, u.ws, s))) return rc;
        if ((rc = union_relabel(u.dG, G, am.m.cvtx, am.m.n_cvtx, am.m.cblk, u.ws.mmap, s))) return rc;
        hipLaunchKernelGGL(k_store_C, dim3((G + 63) / 64), dim3(64), 0, s, (const GDev *)u.dG, G, (int)ACT_COMPACT,
                           (const int *)u.ws.gC, u.Cdev);
        SBP_LAUNCH_CHECK();
    }
    for (int g = 0; g < G; ++g) {
        GraphRun &r = *runs[g];
        if (r.action == ACT_MERGE) ++r.phase_ctr;
    }
    return 0;
}

// The graph's sweep goes on in the same step when what comes next in it is
// another hub or batch: that needs only the blockmodel after the one before,
// no host decision.  Takes the step (as advance would) and returns true.
bool continue_sweep(GraphRun &r) {
    if (!g_batches_in_step || r.phase != GraphRun::MCMC || r.action != ACT_SWEEP) return false;
    if (r.hub_i >= 0) {  // the next hub, else the first batch
        if (++r.hub_i >= r.nh) {
            r.hub_i = -1;
            r.batch = 0;
        }
        return true;
    }
    const int nb = std::max(1, std::min(r.p.n_batches, r.g.n));
    if (r.batch + 1 < nb) {
        ++r.batch;
        return true;
    }
    return false;
}

int engine_step(sbp_engine *eng, int *active_out) {
    hipStream_t s = eng->s;
    UnionLayout &u = eng->u;
    const int G = (int)eng->active.size();
    if (G == 0) {
        if (active_out) *active_out = 0;
        return 0;
    }
    int rc;
    // 1-3: layout, counts, rebuild, DL
    StepState st;
    if ((rc = step_build(eng, eng->active, st, true))) return rc;
    // 4: read back
    eng->h_dl.resize(G);
    eng->h_C.resize(G);
    SBP_HIP_CHECK(hipMemcpyAsync(eng->h_dl.data(), u.ws.dl, G * sizeof(double), hipMemcpyDeviceToHost, s));
    std::vector<int> cd(eng->maxG);
    SBP_HIP_CHECK(hipMemcpyAsync(cd.data(), u.Cdev, eng->maxG * sizeof(int), hipMemcpyDeviceToHost, s));
    SBP_HIP_CHECK(hipStreamSynchronize(s));
    // 5: advance every graph
    for (int g = 0; g < G; ++g) {
        GraphRun &r = *eng->active[g];
        advance(eng, r, eng->h_dl[g], cd[r.eslot]);
    }
    // 6: actions against the blockmodel built above (same layout)
    if ((rc = step_act(eng, eng->active, st))) return rc;
    // 7: the further hubs and batches of the sweeps this step began, each
    // against a blockmodel rebuilt after the one before, with no host round trip
    for (;;) {
        std::vector<GraphRun *> more;
        for (GraphRun *r : eng->active)
            if (continue_sweep(*r)) more.push_back(r);
        if (more.empty()) break;
        StepState st2;
        if ((rc = step_build(eng, more, st2, false))) return rc;
        if ((rc = step_act(eng, more, st2))) return rc;
    }
    // host copy of block counts for graphs that loaded a stored assignment
    for (int g = 0; g < G; ++g) {
        GraphRun &r = *eng->active[g];
        if (r.phase == GraphRun::PRE_MERGE && r.action == ACT_NONE) {
            hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, u.Cdev + r.eslot, r.C);
        }
    }
    // retire finished graphs
    std::vector<GraphRun *> keep;
    for (GraphRun *r : eng->active) {
        if (r->phase == GraphRun::DONE) {
            eng->finished.push_back(r);
        } else {
            keep.push_back(r);
        }
    }
    if (keep.size() != eng->active.size()) {
        SBP_HIP_CHECK(hipStreamSynchronize(s));  // final copies done before the pool is reused
        for (GraphRun *r : eng->active)
            if (r->phase == GraphRun::DONE) {
                pool_free(eng, r->pool_off, r->pool_bytes);
                eng->free_slots.push_back(r->eslot);
                eng->usedV -= r->g.n;
                eng->usedE -= r->g.e;
                std::lock_guard<std::mutex> lk(g_trace_mu);
                g_traces[r->tag] = {r->trace, r->trace_dl};
            }
    }
    eng->active.swap(keep);
    if (active_out) *active_out = (int)eng->active.size();
    return 0;
}

}  // namespace
}  // namespace sbp

// ====================================================================== C-ABI
using namespace sbp;

extern "C" {

const char *sbp_last_error(void) { return sbp::g_err.c_str(); }

size_t sbp_blockmodel_bytes(int32_t n, int32_t e, int32_t C) {
    if (n < 1 || C < 1 || e < 0) return 0;
    return bm_layout(nullptr, n, e, C).bytes;
}

size_t sbp_workspace_bytes(int32_t op, int32_t n, int32_t e, int32_t C) {
    (void)op;
    (void)C;
    if (n < 1 || e < 0) return 0;
    return single_layout(nullptr, 0, n, e).bytes;
}

int sbp_validate_graph(const sbp_graph *g, void *ws, size_t ws_bytes, void *stream) {
    int rc;
    if ((rc = check_graph_args(g))) return rc;
    hipStream_t s = (hipStream_t)stream;
    SingleWS w = single_layout(ws, ws_bytes, g->n, g->e);
    if (!ws || ws_bytes < w.bytes) return fail(SBP_E_SPACE, "workspace too small");
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, w.u.flags, 0);
    hipLaunchKernelGGL(k_validate, dim3(grid_for(g->n + 1, BLK, 4096)), dim3(BLK), 0, s, g->out_ptr, g->out_idx,
                       g->in_ptr, g->n, g->e, w.u.flags);
    hipLaunchKernelGGL(k_validate, dim3(grid_for(g->n + 1, BLK, 4096)), dim3(BLK), 0, s, g->in_ptr, g->in_idx,
                       g->out_ptr, g->n, g->e, w.u.flags);
    SBP_LAUNCH_CHECK();
    int flags = 0;
    SBP_HIP_CHECK(hipMemcpyAsync(&flags, w.u.flags, sizeof(int), hipMemcpyDeviceToHost, s));
    SBP_HIP_CHECK(hipStreamSynchronize(s));
    if (flags & 1) return fail(SBP_E_GRAPH, "malformed CSR/CSC arrays");
    if (flags & 2) return fail(SBP_E_LIMIT, "a vertex has more edge ends than SBP_MAX_DEGREE");
    return 0;
}

size_t sbp_graph_workspace_bytes(int32_t n, int32_t e) {
    if (n < 1 || e < 0) return 0;
    return single_layout(nullptr, 0, n, e).bytes;
}

int sbp_graph_from_edges(int32_t n, int32_t e, const int32_t *src, const int32_t *dst, int32_t *out_ptr,
                         int32_t *out_idx, int32_t *in_ptr, int32_t *in_idx, void *ws, size_t ws_bytes,
                         void *stream) {
    if (n < 1 || e < 0 || !out_ptr || !in_ptr || (e > 0 && (!src || !dst || !out_idx || !in_idx)))
        return fail(SBP_E_ARG, "bad arguments");
    if (n >= (1 << 30) || e >= (1 << 30)) return fail(SBP_E_LIMIT, "n and e must be below 2^30");
    SingleWS w = single_layout(ws, ws_bytes, n, e);
    if (!ws || ws_bytes < w.bytes) return fail(SBP_E_SPACE, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, w.u.flags, 0);
    SBP_LAUNCH_CHECK();
    int rc = graph_from_edges(n, e, src, dst, out_ptr, out_idx, in_ptr, in_idx, w.u.ws, w.u.bm.nnz, w.u.flags, s);
    if (rc) return rc;
    int flag = 0;
    SBP_HIP_CHECK(hipMemcpyAsync(&flag, w.u.flags, sizeof(int), hipMemcpyDeviceToHost, s));
    SBP_HIP_CHECK(hipStreamSynchronize(s));
    return flag ? fail(SBP_E_GRAPH, "edge endpoint outside [0, n)") : 0;
}

int sbp_check_labels(int32_t n, const int32_t *assign, int32_t C, void *ws, size_t ws_bytes, void *stream) {
    if (n < 1 || !assign || C < 1) return fail(SBP_E_ARG, "bad arguments");
    if (!ws || ws_bytes < 256) return fail(SBP_E_SPACE, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    int *flag = (int *)ws;
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, flag, 0);
    hipLaunchKernelGGL(k_check_labels, dim3(grid_for(n, BLK, 4096)), dim3(BLK), 0, s, assign, n, C, flag);
    SBP_LAUNCH_CHECK();
    int h = 0;
    SBP_HIP_CHECK(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    SBP_HIP_CHECK(hipStreamSynchronize(s));
    return h ? fail(SBP_E_LABEL, "label outside [0, C)") : 0;
}

int sbp_build_blockmodel(const sbp_graph *g, const int32_t *assign, int32_t C, void *bm, size_t bm_bytes, void *ws,
                         size_t ws_bytes, void *stream) {
    int rc;
    if ((rc = check_graph_args(g))) return rc;
    if (!assign || !bm || C < 1 || C > g->n) return fail(SBP_E_ARG, "bad assignment, blockmodel or C");
    BMView bv = bm_layout(bm, g->n, g->e, C);
    if (bm_bytes < bv.bytes) return fail(SBP_E_SPACE, "blockmodel storage too small");
    hipStream_t s = (hipStream_t)stream;
    GDev d = gdev_of(g, (int *)assign, C);
    if (bv.dense) return dense_build(d, bv.d, bv.delta, s);
    SingleWS w = single_layout(ws, ws_bytes, g->n, g->e);
    if (!ws || ws_bytes < w.bytes) return fail(SBP_E_SPACE, "workspace too small");
    return build_one(d, w.u, bv, s);
}

int sbp_blockmodel_coo(const sbp_graph *g, int32_t C, const void *bm, int32_t *rows, int32_t *cols, int32_t *vals,
                       int32_t *dout, int32_t *din, int64_t *nnz, void *stream) {
    int rc;
    if ((rc = check_graph_args(g))) return rc;
    if (!bm || !rows || !cols || !vals || !dout || !din || !nnz || C < 1) return fail(SBP_E_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    BMView bv = bm_layout((void *)bm, g->n, g->e, C);
    if (bv.dense) {
        hipLaunchKernelGGL(k_dense_coo, dim3(1), dim3(64), 0, s, bv.d.M, bv.d.dout, bv.d.din, C, rows, cols, vals,
                           dout, din, bv.spare);
        SBP_LAUNCH_CHECK();
        long long k = 0;
        SBP_HIP_CHECK(hipMemcpyAsync(&k, bv.spare, sizeof(long long), hipMemcpyDeviceToHost, s));
        SBP_HIP_CHECK(hipStreamSynchronize(s));
        *nnz = k;
        return 0;
    }
    long long h = 0;
    SBP_HIP_CHECK(hipMemcpyAsync(&h, bv.sp.nnz, sizeof(long long), hipMemcpyDeviceToHost, s));
    SBP_HIP_CHECK(hipStreamSynchronize(s));
    hipLaunchKernelGGL(k_sparse_rows, dim3(grid_for(C, BLK, 4096)), dim3(BLK), 0, s, bv.sp.rptr, C, rows);
    SBP_LAUNCH_CHECK();
    if (h > 0) {
        SBP_HIP_CHECK(hipMemcpyAsync(cols, bv.sp.rcol, h * 4, hipMemcpyDeviceToDevice, s));
        SBP_HIP_CHECK(hipMemcpyAsync(vals, bv.sp.rval, h * 4, hipMemcpyDeviceToDevice, s));
    }
    SBP_HIP_CHECK(hipMemcpyAsync(dout, bv.sp.dout, (size_t)C * 4, hipMemcpyDeviceToDevice, s));
    SBP_HIP_CHECK(hipMemcpyAsync(din, bv.sp.din, (size_t)C * 4, hipMemcpyDeviceToDevice, s));
    SBP_HIP_CHECK(hipStreamSynchronize(s));
    *nnz = h;
    return 0;
}

int sbp_description_length(const sbp_graph *g, int32_t C, const void *bm, double *dl, void *stream) {
    int rc;
    if ((rc = check_graph_args(g))) return rc;
    if (!bm || !dl || C < 1) return fail(SBP_E_ARG, "bad arguments");
    BMView bv = bm_layout((void *)bm, g->n, g->e, C);
    hipLaunchKernelGGL(k_copy_dl, dim3(1), dim3(1), 0, (hipStream_t)stream, (const double *)bv.dl, dl);
    SBP_LAUNCH_CHECK();
    return 0;
}

int sbp_nodal_sweep(const sbp_graph *g, int32_t *assign, int32_t C, void *bm, size_t bm_bytes,
                    const sbp_sweep_params *p, sbp_sweep_stats *stats, const sbp_sweep_trace *trace, void *ws,
                    size_t ws_bytes, void *stream) {
    int rc;
    if ((rc = check_sweep_args(g, assign, C, bm, p))) return rc;
    BMView bv = bm_layout(bm, g->n, g->e, C);
    if (bm_bytes < bv.bytes) return fail(SBP_E_SPACE, "blockmodel storage too small");
    SingleWS w = single_layout(ws, ws_bytes, g->n, g->e);
    if (!ws || ws_bytes < w.bytes) return fail(SBP_E_SPACE, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    sbp_sweep_stats_dev *st = stats ? (sbp_sweep_stats_dev *)stats : w.stats;
    if (!bv.dense) {  // the dense tier's first batch starts the totals itself
        hipLaunchKernelGGL(k_zero_stats, dim3(1), dim3(1), 0, s, st);
        SBP_LAUNCH_CHECK();
    }
    const SweepTraceDev tr = trace_of(trace);
    GDev d = sweep_desc(g, assign, C, p);
    if (bv.dense) {
        DenseScratch ds{};
        HubScratch hs{};
        dense_scratch_of(w, ds, hs);
        return dense_sweep(d, bv, ds, p->n_hubs, hs, tr, st, s);
    }
    SweepTraceDev trs = tr;
    // sparse tier: hub list, then per batch: evaluate + apply, rebuild
    trs.status = w.status;
    if (!trs.dS) trs.dS = w.dS;
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, w.u.hub_count, 0);
    hipLaunchKernelGGL(k_hub_list, dim3(grid_for(g->n, BLK, 4096)), dim3(BLK), 0, s, g->out_ptr, g->in_ptr, g->n, w.hub,
                       w.u.hub_count);
    SBP_LAUNCH_CHECK();
    int n_hub = 0;
    SBP_HIP_CHECK(hipMemcpyAsync(&n_hub, w.u.hub_count, sizeof(int), hipMemcpyDeviceToHost, s));
    SBP_HIP_CHECK(hipStreamSynchronize(s));
    d.hub = w.hub;
    d.n_hub = n_hub;
    // one batch against the blockmodel of the current labels, then the rebuild
    const bool tabled = (long long)C <= g_table_max_c && (long long)C * C <= w.u.table_ints;
    auto run_batch = [&](const GDev &db0) -> int {
        GDev db = db0;
        if (tabled) db.mdense = w.u.tables;
        std::vector<GDev> hG{db};
        HostMeta hm;
        plan_step(hG, hm);
        int rc2;
        if ((rc2 = upload_step(hG, hm, w.u, s))) return rc2;
        SparseBM sbm = bv.sp;
        if (tabled && (rc2 = union_lookup_tables(w.u.dG, 1, 1, sbm, s))) return rc2;
        if ((rc2 = union_sweep(w.u.dG, hm.m, sbm, w.u.ws, trs, s))) return rc2;
        GDev d2 = db;
        d2.action = ACT_NONE;
        if ((rc2 = build_one(d2, w.u, bv, s))) return rc2;
        const int nblk = std::max(1, std::min(dense_workgroups(), (int)((g->n / db.n_batches + 255) / 256)));
        hipLaunchKernelGGL(k_sweep_stats_part, dim3(nblk), dim3(256), 0, s, (const signed char *)w.status,
                           (const double *)trs.dS, g->n, db.batch, db.n_batches, db.skip, w.stats_part, w.sum_part);
        hipLaunchKernelGGL(k_sweep_stats_final, dim3(1), dim3(64), 0, s, (const long long *)w.stats_part,
                           (const double *)w.sum_part, nblk, (const double *)bv.dl, st);
        SBP_LAUNCH_CHECK();
        return 0;
    };
    // hybrid sweep (R21): the hubs one at a time, each a batch of its own
    // ({v : v mod n = hub}) against the blockmodel rebuilt after the one
    // before; the batches then skip them (hub ranks in the dense tier's
    // decision array, unused on this tier)
    if (p->n_hubs > 0) {
        std::vector<int> op(g->n + 1), ip(g->n + 1);
        SBP_HIP_CHECK(hipMemcpyAsync(op.data(), g->out_ptr, (size_t)(g->n + 1) * 4, hipMemcpyDeviceToHost, s));
        SBP_HIP_CHECK(hipMemcpyAsync(ip.data(), g->in_ptr, (size_t)(g->n + 1) * 4, hipMemcpyDeviceToHost, s));
        SBP_HIP_CHECK(hipStreamSynchronize(s));
        std::vector<int> ord(g->n), rank(g->n, 0);
        for (int v = 0; v < g->n; ++v) ord[v] = v;
        auto deg = [&](int v) { return (op[v + 1] - op[v]) + (ip[v + 1] - ip[v]); };
        std::partial_sort(ord.begin(), ord.begin() + p->n_hubs, ord.end(), [&](int a, int c) {
            return deg(a) != deg(c) ? deg(a) > deg(c) : a < c;
        });
        for (int i = 0; i < p->n_hubs; ++i) rank[ord[i]] = i + 1;
        SBP_HIP_CHECK(hipMemcpyAsync(w.nb_dense, rank.data(), (size_t)g->n * 4, hipMemcpyHostToDevice, s));
        for (int i = 0; i < p->n_hubs; ++i) {
            GDev dh = d;
            dh.n_batches = g->n;
            dh.batch = ord[i];
            if ((rc = run_batch(dh))) return rc;
        }
        SBP_HIP_CHECK(hipStreamSynchronize(s));  // the host rank array is released
        d.skip = w.nb_dense;
    }
    for (int b = 0; b < d.n_batches; ++b) {
        d.batch = b;
        if ((rc = run_batch(d))) return rc;
    }
    return 0;
}

int sbp_nodal_sweep_static(const sbp_graph *g, int32_t *assign, int32_t C, void *bm, size_t bm_bytes,
                           const sbp_sweep_params *p, sbp_sweep_stats *stats, const sbp_sweep_trace *trace,
                           void *stream) {
    int rc;
    if ((rc = check_sweep_args(g, assign, C, bm, p))) return rc;
    if (C > SBP_DENSE_MAX_C)
        return fail(SBP_E_ARG, "the allocation-free sweep runs on the dense tier only (C <= 64)");
    if (p->n_hubs != 0) return fail(SBP_E_ARG, "the allocation-free sweep has no hub pass (n_hubs must be 0)");
    if (g->n > SBP_STATIC_MAX_VERTICES)
        return fail(SBP_E_LIMIT, "the allocation-free sweep takes at most SBP_STATIC_MAX_VERTICES vertices");
    BMView bv = bm_layout(bm, g->n, g->e, C);
    if (bm_bytes < bv.bytes) return fail(SBP_E_SPACE, "blockmodel storage too small");
    StaticScratch sc{};
    if ((rc = static_scratch(sc))) return rc;
    hipStream_t s = (hipStream_t)stream;
    DenseScratch ds{};
    ds.nwg = std::min(dense_workgroups(), STATIC_MAX_WGS);
    ds.nb = sc.nb;
    ds.stats_part = sc.stats_part;
    ds.sum_part = sc.sum_part;
    HubScratch hs{};
    return dense_sweep(sweep_desc(g, assign, C, p), bv, ds, 0, hs, trace_of(trace),
                       stats ? (sbp_sweep_stats_dev *)stats : sc.stats, s);
}

int sbp_sweep_graph_create(const sbp_graph *g, int32_t *assign, int32_t C, void *bm, size_t bm_bytes,
                           const sbp_sweep_params *p, uint32_t *sweep_index, sbp_sweep_stats *stats, void *ws,
                           size_t ws_bytes, sbp_sweep_graph **out) {
    int rc;
    if (!out) return fail(SBP_E_ARG, "null output handle");
    *out = nullptr;
    if ((rc = check_sweep_args(g, assign, C, bm, p))) return rc;
    if (!sweep_index || !stats) return fail(SBP_E_ARG, "the sweep index and the statistics record are required");
    if (C > SBP_DENSE_MAX_C) return fail(SBP_E_ARG, "a captured sweep runs on the dense tier only (C <= 64)");
    BMView bv = bm_layout(bm, g->n, g->e, C);
    if (bm_bytes < bv.bytes) return fail(SBP_E_SPACE, "blockmodel storage too small");
    SingleWS w = single_layout(ws, ws_bytes, g->n, g->e);
    if (!ws || ws_bytes < w.bytes) return fail(SBP_E_SPACE, "workspace too small");
    DenseScratch ds{};
    HubScratch hs{};
    dense_scratch_of(w, ds, hs);
    GDev d = sweep_desc(g, assign, C, p);
    d.sweep_dev = sweep_index;
    // capture on a private stream of the default priority, so that the
    // caller's stream (possibly the legacy null stream) is never in capture
    hipStream_t cs = nullptr;
    SBP_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = dense_sweep(d, bv, ds, p->n_hubs, hs, trace_of(nullptr), (sbp_sweep_stats_dev *)stats, cs);
        const hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (!rc && e2 != hipSuccess) rc = fail(SBP_E_HIP, std::string("stream capture: ") + hipGetErrorString(e2));
        if (!rc && (e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess)
            rc = fail(SBP_E_HIP, std::string("graph instantiation: ") + hipGetErrorString(e));
    } else {
        rc = fail(SBP_E_HIP, std::string("stream capture: ") + hipGetErrorString(e));
    }
    (void)hipStreamDestroy(cs);
    if (rc) {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    *out = new sbp_sweep_graph{graph, exec, dev};
    return 0;
}

int sbp_sweep_graph_launch(sbp_sweep_graph *h, void *stream) {
    if (!h) return fail(SBP_E_ARG, "null graph handle");
    int dev = 0;
    SBP_HIP_CHECK(hipGetDevice(&dev));
    if (dev != h->dev) return fail(SBP_E_ARG, "the graph was captured on another device");
    SBP_HIP_CHECK(hipGraphLaunch(h->exec, (hipStream_t)stream));
    return 0;
}

int sbp_sweep_graph_destroy(sbp_sweep_graph *h) {
    if (!h) return 0;
    const hipError_t a = hipGraphExecDestroy(h->exec), b = hipGraphDestroy(h->graph);
    delete h;
    if (a != hipSuccess || b != hipSuccess) return fail(SBP_E_HIP, "graph destruction failed");
    return 0;
}

int sbp_merge_scores(const sbp_graph *g, const int32_t *assign, int32_t C, const void *bm, const sbp_merge_params *p,
                     int32_t *partner, double *dS, double *dS_local, void *ws, size_t ws_bytes, void *stream) {
    int rc;
    if ((rc = check_graph_args(g))) return rc;
    if (!assign || !bm || !p || !partner || !dS || C < 1 || C > g->n || p->proposals < 1 || p->eps < 0)
        return fail(SBP_E_ARG, "bad merge arguments");
    BMView bv = bm_layout((void *)bm, g->n, g->e, C);
    SingleWS w = single_layout(ws, ws_bytes, g->n, g->e);
    if (!ws || ws_bytes < w.bytes) return fail(SBP_E_SPACE, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    GDev d = gdev_of(g, (int *)assign, C);
    d.seed = p->seed;
    d.phase = p->phase;
    d.proposals = p->proposals;
    d.eps = p->eps;
    d.action = ACT_MERGE;
    double *dsl = dS_local ? dS_local : w.u.dSl;
    if (bv.dense) return dense_merge_scores(d, bv.d, partner, dS, dsl, s);
    std::vector<GDev> hG{d};
    HostMeta hm;
    plan_step(hG, hm);
    if ((rc = upload_step(hG, hm, w.u, s))) return rc;
    return union_merge_scores(w.u.dG, hm.m, bv.sp, partner, dS, dsl, s);
}

int sbp_merge_apply(int32_t C, const int32_t *partner, const double *dS_local, int32_t n_merges, int32_t *map,
                    int32_t *C_new, void *ws, size_t ws_bytes, void *stream) {
    if (C < 1 || !partner || !dS_local || !map || !C_new || n_merges < 0) return fail(SBP_E_ARG, "bad arguments");
    SingleWS w = single_layout(ws, ws_bytes, C, 1);
    if (!ws || ws_bytes < w.bytes) return fail(SBP_E_SPACE, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    int rc;
    sbp_graph fake{};
    fake.n = C;
    GDev d = gdev_of(&fake, nullptr, C);
    d.merges = n_merges;
    d.action = ACT_MERGE;
    std::vector<GDev> hG{d};
    HostMeta hm;
    plan_step(hG, hm);
    if ((rc = upload_step(hG, hm, w.u, s))) return rc;
    if ((rc = union_merge_apply(w.u.dG, hm.m, partner, dS_local, w.u.ws, s))) return rc;
    SBP_HIP_CHECK(hipMemcpyAsync(map, w.u.ws.mmap, (size_t)C * 4, hipMemcpyDeviceToDevice, s));
    int h = 0;
    SBP_HIP_CHECK(hipMemcpyAsync(&h, w.u.ws.gC, sizeof(int), hipMemcpyDeviceToHost, s));
    SBP_HIP_CHECK(hipStreamSynchronize(s));
    *C_new = h;
    return 0;
}

int sbp_relabel(int32_t n, int32_t *assign, const int32_t *map, void *stream) {
    if (n < 1 || !assign || !map) return fail(SBP_E_ARG, "bad arguments");
    hipLaunchKernelGGL(k_relabel_map, dim3(grid_for(n, BLK, 4096)), dim3(BLK), 0, (hipStream_t)stream, assign, map, n);
    SBP_LAUNCH_CHECK();
    return 0;
}

int sbp_compact(int32_t n, int32_t *assign, int32_t C, int32_t *C_new, void *ws, size_t ws_bytes, void *stream) {
    if (n < 1 || !assign || C < 1 || !C_new) return fail(SBP_E_ARG, "bad arguments");
    SingleWS w = single_layout(ws, ws_bytes, std::max(n, C), 1);
    if (!ws || ws_bytes < w.bytes) return fail(SBP_E_SPACE, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    int rc;
    sbp_graph fake{};
    fake.n = n;
    GDev d = gdev_of(&fake, assign, C);
    d.action = ACT_COMPACT;
    std::vector<GDev> hG{d};
    HostMeta hm;
    plan_step(hG, hm);
    if ((rc = upload_step(hG, hm, w.u, s))) return rc;
    if ((rc = union_compact(w.u.dG, hm.m, w.u.ws, s))) return rc;
    if ((rc = union_relabel(w.u.dG, 1, hm.m.cvtx, hm.m.n_cvtx, hm.m.cblk, w.u.ws.mmap, s))) return rc;
    int h = 0;
    SBP_HIP_CHECK(hipMemcpyAsync(&h, w.u.ws.gC, sizeof(int), hipMemcpyDeviceToHost, s));
    SBP_HIP_CHECK(hipStreamSynchronize(s));
    *C_new = h;
    return 0;
}

// ------------------------------------------------------------------ engine API
size_t sbp_engine_graph_bytes(int32_t n, int32_t e) { return graph_bytes(n, e); }

size_t sbp_engine_workspace_bytes(int64_t max_vertices, int64_t max_edges, int32_t max_graphs) {
    if (max_vertices < 1 || max_edges < 0 || max_graphs < 1) return 0;
    Arena a = Arena::measure();
    union_layout(a, max_vertices, max_edges, max_graphs);
    return a.used + al(pool_bound(max_vertices, max_edges, max_graphs));
}

int sbp_engine_create(void *ws, size_t ws_bytes, int64_t max_vertices, int64_t max_edges, int32_t max_graphs,
                      void *stream, sbp_engine **out) {
    if (!out || max_vertices < 1 || max_edges < 0 || max_graphs < 1) return fail(SBP_E_ARG, "bad engine arguments");
    if (max_vertices >= (1LL << 30) || max_edges >= (1LL << 30)) return fail(SBP_E_LIMIT, "engine capacity too large");
    const size_t need = sbp_engine_workspace_bytes(max_vertices, max_edges, max_graphs);
    if (!ws || ws_bytes < need) return fail(SBP_E_SPACE, "engine workspace too small");
    sbp_engine *eng = new sbp_engine();
    eng->s = (hipStream_t)stream;
    eng->base = (char *)ws;
    eng->bytes = ws_bytes;
    eng->maxV = max_vertices;
    eng->maxE = max_edges;
    eng->maxG = max_graphs;
    Arena a(ws, ws_bytes);
    eng->u = union_layout(a, max_vertices, max_edges, max_graphs);
    fill_ftab(eng->u.ftab, eng->u.ftab_max, eng->s);
    SBP_LAUNCH_CHECK();
    const size_t pool_off = a.used;
    eng->pool_bytes = ws_bytes - pool_off;
    eng->free_list.push_back({pool_off, eng->pool_bytes});
    for (int i = max_graphs - 1; i >= 0; --i) eng->free_slots.push_back(i);
    *out = eng;
    return 0;
}

int sbp_engine_admit(sbp_engine *eng, const sbp_graph *g, const sbp_partition_params *p, int32_t *assign_out,
                     int32_t C_init, int64_t tag) {
    int rc;
    if (!eng || !p || !assign_out) return fail(SBP_E_ARG, "bad arguments");
    if ((rc = check_graph_args(g))) return rc;
    if (p->merge_proposals < 1 || p->eps < 0 || !(p->beta > 0) || p->n_batches < 1 || p->max_iters < 0 ||
        p->n_hubs < 0 || !(p->merge_rate >= 0 && p->merge_rate <= 1))
        return fail(SBP_E_ARG, "bad partition parameters");
    if (C_init < 0 || C_init > g->n) return fail(SBP_E_ARG, "bad initial block count");
    if ((int)eng->active.size() >= eng->maxG || eng->usedV + g->n > eng->maxV || eng->usedE + g->e > eng->maxE ||
        eng->free_slots.empty())
        return fail(SBP_E_SPACE, "engine full");
    const size_t bytes = graph_bytes(g->n, g->e);
    size_t off = 0;
    if (!pool_alloc(eng, bytes, off)) return fail(SBP_E_SPACE, "engine pool full");
    hipStream_t s = eng->s;
    GraphRun *r = new GraphRun();
    r->tag = tag;
    r->g = *g;
    r->p = *p;
    r->lab = assign_out;
    r->pool_off = off;
    r->pool_bytes = bytes;
    char *b = eng->base + off;
    for (int k = 0; k < 3; ++k) {
        r->slot_lab[k] = (int *)b;
        b += al((size_t)g->n * 4);
    }
    r->hub_rank = (int *)b;
    b += al((size_t)g->n * 4);
    r->hub = (int *)b;
    r->nh = std::min(p->n_hubs, g->n);
    if (r->nh > 0) {
        // the hubs of a hybrid sweep: degree (out + in ends) descending, ties by id
        std::vector<int> op(g->n + 1), ip(g->n + 1);
        SBP_HIP_CHECK(hipMemcpyAsync(op.data(), g->out_ptr, (size_t)(g->n + 1) * 4, hipMemcpyDeviceToHost, s));
        SBP_HIP_CHECK(hipMemcpyAsync(ip.data(), g->in_ptr, (size_t)(g->n + 1) * 4, hipMemcpyDeviceToHost, s));
        SBP_HIP_CHECK(hipStreamSynchronize(s));
        std::vector<int> ord(g->n);
        for (int v = 0; v < g->n; ++v) ord[v] = v;
        auto deg = [&](int v) { return (op[v + 1] - op[v]) + (ip[v + 1] - ip[v]); };
        std::partial_sort(ord.begin(), ord.begin() + r->nh, ord.end(), [&](int a, int c) {
            return deg(a) != deg(c) ? deg(a) > deg(c) : a < c;
        });
        r->hub_order.assign(ord.begin(), ord.begin() + r->nh);
        std::vector<int> rank(g->n, 0);
        for (int i = 0; i < r->nh; ++i) rank[r->hub_order[i]] = i + 1;
        SBP_HIP_CHECK(hipMemcpyAsync(r->hub_rank, rank.data(), (size_t)g->n * 4, hipMemcpyHostToDevice, s));
        SBP_HIP_CHECK(hipStreamSynchronize(s));
    }
    // hub list (vertices with more than SBP_LEAF_MAX edge ends)
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, eng->u.hub_count, 0);
    hipLaunchKernelGGL(k_hub_list, dim3(grid_for(g->n, BLK, 4096)), dim3(BLK), 0, s, g->out_ptr, g->in_ptr, g->n,
                       r->hub, eng->u.hub_count);
    if (C_init == 0) hipLaunchKernelGGL(k_iota, dim3(grid_for(g->n, BLK, 4096)), dim3(BLK), 0, s, assign_out, g->n);
    SBP_LAUNCH_CHECK();
    int nh = 0;
    SBP_HIP_CHECK(hipMemcpyAsync(&nh, eng->u.hub_count, sizeof(int), hipMemcpyDeviceToHost, s));
    SBP_HIP_CHECK(hipStreamSynchronize(s));
    r->n_hub = nh;
    r->eslot = eng->free_slots.back();
    eng->free_slots.pop_back();
    r->C = C_init == 0 ? g->n : C_init;
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, eng->u.Cdev + r->eslot, r->C);
    SBP_LAUNCH_CHECK();
    r->phase = GraphRun::START;
    eng->usedV += g->n;
    eng->usedE += g->e;
    eng->active.push_back(r);
    return 0;
}

int sbp_engine_step(sbp_engine *eng, int32_t *active) {
    if (!eng) return fail(SBP_E_ARG, "null engine");
    return engine_step(eng, active);
}

int sbp_engine_poll(sbp_engine *eng, int64_t *tag, int32_t *C, double *dl) {
    if (!eng || eng->finished.empty()) return 0;
    GraphRun *r = eng->finished.front();
    eng->finished.erase(eng->finished.begin());
    if (tag) *tag = r->tag;
    if (C) *C = r->final_C;
    if (dl) *dl = r->final_dl;
    delete r;
    return 1;
}

int sbp_engine_destroy(sbp_engine *eng) {
    if (!eng) return 0;
    for (GraphRun *r : eng->active) delete r;
    for (GraphRun *r : eng->finished) delete r;
    delete eng;
    return 0;
}

size_t sbp_partition_workspace_bytes(int32_t n_graphs, const int32_t *n, const int32_t *e) {
    if (n_graphs < 1 || !n || !e) return 0;
    long long V = 0, E = 0;
    for (int i = 0; i < n_graphs; ++i) {
        V += n[i];
        E += e[i];
    }
    return sbp_engine_workspace_bytes(V, E, n_graphs);
}

int sbp_partition_batch(int32_t n_graphs, const sbp_graph *graphs, const sbp_partition_params *params,
                        int32_t *const *assign_out, int32_t *C_out, double *dl_out, void *ws, size_t ws_bytes,
                        void *stream) {
    if (n_graphs < 1 || !graphs || !params || !assign_out || !C_out || !dl_out) return fail(SBP_E_ARG, "bad arguments");
    long long V = 0, E = 0;
    for (int i = 0; i < n_graphs; ++i) {
        V += graphs[i].n;
        E += graphs[i].e;
    }
    sbp_engine *eng = nullptr;
    int rc = sbp_engine_create(ws, ws_bytes, V, E, n_graphs, stream, &eng);
    if (rc) return rc;
    for (int i = 0; i < n_graphs && !rc; ++i) rc = sbp_engine_admit(eng, &graphs[i], &params[i], assign_out[i], 0, i);
    int active = 1;
    while (!rc && active > 0) rc = sbp_engine_step(eng, &active);
    if (!rc) {
        int64_t tag;
        int C;
        double dl;
        while (sbp_engine_poll(eng, &tag, &C, &dl)) {
            C_out[tag] = C;
            dl_out[tag] = dl;
        }
    }
    sbp_engine_destroy(eng);
    return rc;
}

int sbp_partition(const sbp_graph *g, const int32_t *assign_in, int32_t C_in, const sbp_partition_params *p,
                  int32_t *assign_out, int32_t *C_out, double *dl_out, void *ws, size_t ws_bytes, void *stream) {
    int rc;
    if ((rc = check_graph_args(g))) return rc;
    if (!p || !assign_out || !C_out || !dl_out) return fail(SBP_E_ARG, "bad arguments");
    sbp_engine *eng = nullptr;
    if ((rc = sbp_engine_create(ws, ws_bytes, g->n, g->e, 1, stream, &eng))) return rc;
    int C0 = 0;
    if (assign_in) {
        if (C_in < 1 || C_in > g->n) {
            sbp_engine_destroy(eng);
            return fail(SBP_E_ARG, "bad C_in");
        }
        hipStream_t s = (hipStream_t)stream;
        if ((rc = sbp_check_labels(g->n, assign_in, C_in, eng->u.flags, 256, stream))) {
            sbp_engine_destroy(eng);
            return rc;
        }
        if (assign_in != assign_out)
            SBP_HIP_CHECK(hipMemcpyAsync(assign_out, assign_in, (size_t)g->n * 4, hipMemcpyDeviceToDevice, s));
        // compact the start in place with the engine's scratch
        std::vector<GDev> hG{gdev_of(g, assign_out, C_in)};
        hG[0].action = ACT_COMPACT;
        HostMeta hm;
        plan_step(hG, hm);
        if (!(rc = upload_step(hG, hm, eng->u, s)) && !(rc = union_compact(eng->u.dG, hm.m, eng->u.ws, s)) &&
            !(rc = union_relabel(eng->u.dG, 1, hm.m.cvtx, hm.m.n_cvtx, hm.m.cblk, eng->u.ws.mmap, s))) {
            SBP_HIP_CHECK(hipMemcpyAsync(&C0, eng->u.ws.gC, sizeof(int), hipMemcpyDeviceToHost, s));
            SBP_HIP_CHECK(hipStreamSynchronize(s));
        }
    }
    if (!rc) rc = sbp_engine_admit(eng, g, p, assign_out, C0, -1);
    int active = 1;
    while (!rc && active > 0) rc = sbp_engine_step(eng, &active);
    if (!rc) {
        int64_t tag;
        if (!sbp_engine_poll(eng, &tag, C_out, dl_out)) rc = fail(SBP_E_ARG, "partition did not finish");
    }
    sbp_engine_destroy(eng);
    return rc;
}

int sbp_tune(const char *key, int64_t value) {
    if (!key) return fail(SBP_E_ARG, "null key");
    if (!strcmp(key, "engine_dense_max_c") && value >= 0 && value <= SBP_DENSE_MAX_C) {
        g_engine_dense_max_c = (int)value;
        return 0;
    }
    if (!strcmp(key, "table_max_c") && value >= 0 && value <= SBP_TABLE_MAX_C) {
        g_table_max_c = (int)value;
        return 0;
    }
    if (!strcmp(key, "table_build_ratio") && value >= 1 && value <= 1024) {
        g_table_ratio = (int)value;
        return 0;
    }
    if (!strcmp(key, "table_build") && value >= 0 && value <= 2) {
        g_table_build = (int)value;
        return 0;
    }
    if (!strcmp(key, "batches_in_step") && (value == 0 || value == 1)) {
        g_batches_in_step = (int)value;
        return 0;
    }
    if (dense_tune(key, (long long)value) == 0) return 0;
    return fail(SBP_E_ARG, std::string("unknown tuning key or value: ") + key);
}

int sbp_profile_enable(int32_t on) {
    if (on < 0) return fail(SBP_E_ARG, "profile stride must be >= 0");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_stride = on;
    for (auto &kv : g_prof) kv.second.calls = 0;  // sampling starts at the next launch
    return 0;
}

int sbp_profile_read(const char *kernel, double *ms, int64_t *launches, int32_t reset) {
    if (!kernel || !ms || !launches) return fail(SBP_E_ARG, "bad arguments");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (strcmp(kernel, "sweep_eval") != 0) return fail(SBP_E_ARG, "unknown kernel name");
    ProfRec &r = g_prof[kernel];
    double total = 0.0;
    for (auto &p : r.ev) {
        SBP_HIP_CHECK(hipEventSynchronize(p.second));
        float t = 0.f;
        SBP_HIP_CHECK(hipEventElapsedTime(&t, p.first, p.second));
        total += t;
    }
    *ms = total;
    *launches = (int64_t)r.ev.size();
    if (reset) {
        for (auto &p : r.ev) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
        r.ev.clear();
    }
    return 0;
}

int sbp_partition_trace(int64_t tag, int64_t *rows, double *dl, int32_t cap) {
    std::lock_guard<std::mutex> lk(g_trace_mu);
    auto it = g_traces.find(tag);
    if (it == g_traces.end()) return 0;
    const auto &tr = it->second;
    const int nrows = (int)tr.second.size();
    const int k = std::min(nrows, (int)cap);
    for (int i = 0; i < k; ++i) {
        for (int j = 0; j < 5; ++j) rows[5 * i + j] = tr.first[5 * i + j];
        dl[i] = tr.second[i];
    }
    g_traces.erase(it);  // read once: a long-lived server does not keep every finished graph's record
    return k;
}

}  // extern "C"
