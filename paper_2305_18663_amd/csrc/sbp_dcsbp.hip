// sbp_dcsbp.hip -- divide-and-conquer SBP (Sec. II-C, Alg. 3) on one GPU.
//
// The vertices are split round robin into s subgraphs (v -> v mod s); each
// induced subgraph is partitioned by the whole method, all of them together
// in one batched engine run (the ranks of Alg. 3 become graphs of one
// launch).  The partial results are then combined pairwise -- every community
// of the second joins the community of the first whose merge changes DL
// least, scored on the blockmodel of the graph the two induce -- while more
// than four remain; the rest are concatenated and the whole method continues
// on the full graph from that assignment.
//
// Induced subgraphs are built on the device: keep flags, an exclusive scan
// for the new ids, per-vertex counts of kept neighbours, scans for the
// pointers, and an emit pass (neighbours stay ascending because the new ids
// keep the order of the old ones).  Partial results live in two n-long arrays
// (global vertex ids and labels), results in list order, so a combined pair
// takes the place of its two parts.
#include <algorithm>
#include <vector>

#include "../../include/sbp.h"
#include "sbp_internal.h"

namespace sbp {

namespace {

constexpr int BLK = 256;

__global__ void k_keep_residue(unsigned char *__restrict__ keep, int n, int s, int r) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) keep[v] = (v % s) == r;
}

// keep[vid[i]] = 1 and lab[vid[i]] = val[i] + off for the listed vertices
__global__ void k_keep_list(unsigned char *__restrict__ keep, int *__restrict__ lab, const int *__restrict__ vid,
                            const int *__restrict__ val, int m, int off) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        keep[vid[i]] = 1;
        lab[vid[i]] = val[i] + off;
    }
}

__global__ void k_zero_u8(unsigned char *__restrict__ p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// flag[v] = keep[v]; kept out- and in-neighbours of kept vertices
__global__ void k_ind_count(sbp_graph g, const unsigned char *__restrict__ keep, int *__restrict__ flag,
                            int *__restrict__ cnt_out, int *__restrict__ cnt_in) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += gridDim.x * blockDim.x) {
        const bool k = keep[v];
        int co = 0, ci = 0;
        if (k) {
            for (int j = g.out_ptr[v]; j < g.out_ptr[v + 1]; ++j) co += keep[g.out_idx[j]];
            for (int j = g.in_ptr[v]; j < g.in_ptr[v + 1]; ++j) ci += keep[g.in_idx[j]];
        }
        flag[v] = k;
        cnt_out[v] = co;
        cnt_in[v] = ci;
    }
}

// The induced CSR/CSC (new ids from the scan of the keep flags), the global
// id of every new vertex, and the labels carried over from glab.
__global__ void k_ind_emit(sbp_graph g, const unsigned char *__restrict__ keep, const long long *__restrict__ sid,
                           const long long *__restrict__ po, const long long *__restrict__ pi, int *__restrict__ s_out_ptr,
                           int *__restrict__ s_out_idx, int *__restrict__ s_in_ptr, int *__restrict__ s_in_idx,
                           int *__restrict__ vid, const int *__restrict__ glab, int *__restrict__ slab) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += gridDim.x * blockDim.x) {
        if (!keep[v]) continue;
        const int i = (int)sid[v];
        long long o = po[v], q = pi[v];
        s_out_ptr[i] = (int)o;
        s_in_ptr[i] = (int)q;
        for (int j = g.out_ptr[v]; j < g.out_ptr[v + 1]; ++j) {
            const int w = g.out_idx[j];
            if (keep[w]) s_out_idx[o++] = (int)sid[w];
        }
        for (int j = g.in_ptr[v]; j < g.in_ptr[v + 1]; ++j) {
            const int w = g.in_idx[j];
            if (keep[w]) s_in_idx[q++] = (int)sid[w];
        }
        vid[i] = v;
        if (glab) slab[i] = glab[v];
    }
}

__global__ void k_ind_tail(int *__restrict__ s_out_ptr, int *__restrict__ s_in_ptr, const long long *__restrict__ tot,
                           int k) {
    s_out_ptr[k] = (int)tot[1];
    s_in_ptr[k] = (int)tot[2];
}

// combined labels: a label of the second result maps to its chosen community
__global__ void k_combine_apply(int *__restrict__ lab, int m, int C1, const int *__restrict__ best) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        const int x = lab[i];
        if (x >= C1) lab[i] = best[x - C1];
    }
}

// assign[vid[i]] = lab[i] + off
__global__ void k_scatter_labels(int *__restrict__ assign, const int *__restrict__ vid, const int *__restrict__ lab,
                                 int m, int off) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) assign[vid[i]] = lab[i] + off;
}

size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

// Workspace of the induced-subgraph builder and the result lists.
struct DcWs {
    unsigned char *keep;
    int *flag, *cnt_out, *cnt_in;
    long long *sid, *po, *pi, *tot;
    void *scan_temp;
    int *sop, *soi, *sip, *sii;  // induced CSR/CSC: [n + s + 1], [e + 1] each
    int *vid_all, *lab_all;      // results in list order [n]
    int *tvid, *tlab, *glab;     // combination scratch [n]
    int *best;                   // [n]
    char *phase;                 // region shared by the batched partition, the builds and the final run
    size_t phase_bytes;
    size_t bytes;
};

DcWs dc_layout(void *base, size_t cap, int n, int e, int s) {
    DcWs w{};
    char *b = (char *)base;
    size_t u = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? b + u : nullptr;
        u += al(bytes > 0 ? bytes : 1);
        return p;
    };
    w.keep = (unsigned char *)take((size_t)n);
    w.flag = (int *)take((size_t)n * 4);
    w.cnt_out = (int *)take((size_t)n * 4);
    w.cnt_in = (int *)take((size_t)n * 4);
    w.sid = (long long *)take(((size_t)n + 1) * 8);
    w.po = (long long *)take(((size_t)n + 1) * 8);
    w.pi = (long long *)take(((size_t)n + 1) * 8);
    w.tot = (long long *)take(4 * 8);
    w.scan_temp = take(scan_temp_bytes((long long)n + 1));
    w.sop = (int *)take(((size_t)n + s + 1) * 4);
    w.sip = (int *)take(((size_t)n + s + 1) * 4);
    w.soi = (int *)take(((size_t)e + 1) * 4);
    w.sii = (int *)take(((size_t)e + 1) * 4);
    w.vid_all = (int *)take((size_t)n * 4);
    w.lab_all = (int *)take((size_t)n * 4);
    w.tvid = (int *)take((size_t)n * 4);
    w.tlab = (int *)take((size_t)n * 4);
    w.glab = (int *)take((size_t)n * 4);
    w.best = (int *)take((size_t)n * 4);
    // the phases run one after another in the same region
    size_t ph = sbp_engine_workspace_bytes(n, e, s);
    ph = std::max(ph, sbp_engine_workspace_bytes(n, e, 1));
    ph = std::max(ph, al(sparse_one_bytes(n, e)) + al((size_t)n * 4 + 256));
    w.phase = take(ph);
    w.phase_bytes = al(ph);
    w.bytes = u;
    (void)cap;
    return w;
}

// Induced subgraph of the kept vertices into sop/soi/sip/sii at the given
// offsets (pointer arrays at pbase, index arrays at ibase); vid[i] = the
// global id of new vertex i; labels from glab into slab when glab is set.
// Returns the vertex and edge counts (one host read).
int induced(const sbp_graph &g, DcWs &w, int pbase, long long ibase, int *vid, const int *glab, int *slab, int &k,
            int &m, hipStream_t s) {
    const int gr = grid_for(g.n, BLK, 4096);
    hipLaunchKernelGGL(k_ind_count, dim3(gr), dim3(BLK), 0, s, g, (const unsigned char *)w.keep, w.flag, w.cnt_out,
                       w.cnt_in);
    SBP_LAUNCH_CHECK();
    int rc;
    if ((rc = scan_exclusive_i32(w.flag, w.sid, g.n, w.tot + 0, w.scan_temp, s))) return rc;
    if ((rc = scan_exclusive_i32(w.cnt_out, w.po, g.n, w.tot + 1, w.scan_temp, s))) return rc;
    if ((rc = scan_exclusive_i32(w.cnt_in, w.pi, g.n, w.tot + 2, w.scan_temp, s))) return rc;
    long long tot[3] = {0, 0, 0};
    SBP_HIP_CHECK(hipMemcpyAsync(tot, w.tot, 3 * sizeof(long long), hipMemcpyDeviceToHost, s));
    SBP_HIP_CHECK(hipStreamSynchronize(s));
    if (tot[1] != tot[2]) return fail(SBP_E_GRAPH, "induced subgraph: CSR and CSC edge counts differ");
    k = (int)tot[0];
    m = (int)tot[1];
    hipLaunchKernelGGL(k_ind_emit, dim3(gr), dim3(BLK), 0, s, g, (const unsigned char *)w.keep,
                       (const long long *)w.sid, (const long long *)w.po, (const long long *)w.pi, w.sop + pbase,
                       w.soi + ibase, w.sip + pbase, w.sii + ibase, vid, glab, slab);
    hipLaunchKernelGGL(k_ind_tail, dim3(1), dim3(1), 0, s, w.sop + pbase, w.sip + pbase, (const long long *)w.tot, k);
    SBP_LAUNCH_CHECK();
    return 0;
}

sbp_graph sub_graph(const DcWs &w, int pbase, long long ibase, int k, int m) {
    sbp_graph h{};
    h.n = k;
    h.e = m;
    h.out_ptr = w.sop + pbase;
    h.out_idx = w.soi + ibase;
    h.in_ptr = w.sip + pbase;
    h.in_idx = w.sii + ibase;
    return h;
}

struct Piece {
    int off, nv, C;  // region [off, off + nv) of vid_all / lab_all
};

}  // namespace
}  // namespace sbp

using namespace sbp;

extern "C" {

size_t sbp_dcsbp_workspace_bytes(int32_t n, int32_t e, int32_t n_sub) {
    if (n < 1 || e < 0 || n_sub < 1 || n_sub > n) return 0;
    return dc_layout(nullptr, 0, n, e, n_sub).bytes;
}

int sbp_dcsbp(const sbp_graph *g, int32_t n_sub, const sbp_partition_params *p, int32_t *assign_out, int32_t *C_out,
              double *dl_out, int32_t *sub_C, void *ws, size_t ws_bytes, void *stream) {
    if (!g || !p || !assign_out || !C_out || !dl_out) return fail(SBP_E_ARG, "bad arguments");
    if (g->n < 1 || n_sub < 1 || n_sub > g->n) return fail(SBP_E_ARG, "n_sub must lie in [1, n]");
    const int n = g->n, e = g->e, s = n_sub;
    DcWs w = dc_layout(ws, ws_bytes, n, e, s);
    if (!ws || ws_bytes < w.bytes) return fail(SBP_E_SPACE, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    int rc;
    // 1: the s induced subgraphs, side by side, then one batched partition
    std::vector<sbp_graph> subs(s);
    std::vector<sbp_partition_params> ps(s, *p);
    std::vector<int32_t *> outs(s);
    std::vector<Piece> R(s);
    int voff = 0;
    long long eoff = 0;
    for (int r = 0; r < s; ++r) {
        hipLaunchKernelGGL(k_keep_residue, dim3(grid_for(n, BLK, 4096)), dim3(BLK), 0, st, w.keep, n, s, r);
        SBP_LAUNCH_CHECK();
        int k = 0, m = 0;
        if ((rc = induced(*g, w, voff + r, eoff, w.vid_all + voff, nullptr, nullptr, k, m, st))) return rc;
        subs[r] = sub_graph(w, voff + r, eoff, k, m);
        ps[r].seed = p->seed + 1 + (uint64_t)r;
        outs[r] = w.lab_all + voff;
        R[r] = Piece{voff, k, 0};
        voff += k;
        eoff += m;
    }
    {
        std::vector<int32_t> Cs(s);
        std::vector<double> dls(s);
        if ((rc = sbp_partition_batch(s, subs.data(), ps.data(), outs.data(), Cs.data(), dls.data(), w.phase,
                                      w.phase_bytes, stream)))
            return rc;
        for (int r = 0; r < s; ++r) {
            R[r].C = Cs[r];
            if (sub_C) sub_C[r] = Cs[r];
            (void)sbp_partition_trace(r, nullptr, nullptr, 0);  // the subgraph runs keep no record
        }
    }
    // 2: pairwise combination while more than four results remain
    while (R.size() > 4) {
        std::vector<Piece> next;
        for (size_t i = 0; i < R.size(); i += 2) {
            if (i + 1 == R.size()) {
                next.push_back(R[i]);
                break;
            }
            const Piece a = R[i], b = R[i + 1];
            hipLaunchKernelGGL(k_zero_u8, dim3(grid_for(n, BLK, 4096)), dim3(BLK), 0, st, w.keep, n);
            hipLaunchKernelGGL(k_keep_list, dim3(grid_for(a.nv, BLK, 4096)), dim3(BLK), 0, st, w.keep, w.glab,
                               (const int *)w.vid_all + a.off, (const int *)w.lab_all + a.off, a.nv, 0);
            hipLaunchKernelGGL(k_keep_list, dim3(grid_for(b.nv, BLK, 4096)), dim3(BLK), 0, st, w.keep, w.glab,
                               (const int *)w.vid_all + b.off, (const int *)w.lab_all + b.off, b.nv, a.C);
            SBP_LAUNCH_CHECK();
            int k = 0, m = 0;
            if ((rc = induced(*g, w, 0, 0, w.tvid, w.glab, w.tlab, k, m, st))) return rc;
            // blockmodel of the pair's graph with the second result's labels after the first's
            GDev d{};
            d.out_ptr = w.sop;
            d.out_idx = w.soi;
            d.in_ptr = w.sip;
            d.in_idx = w.sii;
            d.lab = w.tlab;
            d.n = k;
            d.e = m;
            d.C = a.C + b.C;
            d.n_batches = 1;
            d.eps = 1;
            d.beta = 1.0;
            SparseBM bm{};
            if ((rc = build_sparse_one(d, w.phase, w.phase_bytes, bm, st))) return rc;
            if ((rc = union_combine_choice(bm, a.C, b.C, w.best, st))) return rc;
            hipLaunchKernelGGL(k_combine_apply, dim3(grid_for(k, BLK, 4096)), dim3(BLK), 0, st, w.tlab, k, a.C,
                               (const int *)w.best);
            SBP_LAUNCH_CHECK();
            int32_t Cn = 0;
            if ((rc = sbp_compact(k, w.tlab, a.C, &Cn, w.phase, w.phase_bytes, stream))) return rc;
            // the pair's region is a.off .. a.off + k (the parts are adjacent)
            SBP_HIP_CHECK(hipMemcpyAsync(w.vid_all + a.off, w.tvid, (size_t)k * 4, hipMemcpyDeviceToDevice, st));
            SBP_HIP_CHECK(hipMemcpyAsync(w.lab_all + a.off, w.tlab, (size_t)k * 4, hipMemcpyDeviceToDevice, st));
            next.push_back(Piece{a.off, k, Cn});
        }
        R.swap(next);
    }
    // 3: concatenation, then the whole method on the full graph
    int off = 0;
    for (const Piece &q : R) {
        hipLaunchKernelGGL(k_scatter_labels, dim3(grid_for(q.nv, BLK, 4096)), dim3(BLK), 0, st, assign_out,
                           (const int *)w.vid_all + q.off, (const int *)w.lab_all + q.off, q.nv, off);
        off += q.C;
    }
    SBP_LAUNCH_CHECK();
    return sbp_partition(g, assign_out, off, p, assign_out, C_out, dl_out, w.phase, w.phase_bytes, stream);
}

}  // extern "C"
