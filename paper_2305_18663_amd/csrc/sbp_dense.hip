// sbp_dense.hip -- dense blockmodel tier for C <= 64 blocks (gfx950).
//
// With at most 64 blocks a wave64 lane owns one block t.  M (C x C int32,
// Sec. II-A) and the per-block running sums of e_t. = M_t. + M_.t (the
// proposal tables) live in global memory and are staged in LDS by every
// workgroup of a sweep.  One sweep batch is four launches:
//   eval   -- persistent grid, wave per vertex: neighbour-block histogram in
//             LDS, Philox proposal, DL change over the changed entries of M and
//             the block degrees (Eq. 1-2), Hastings term, accept test (Alg. 2),
//             all against the snapshot taken at the start of the batch;
//   delta  -- every edge with a moved endpoint moves one count from
//             (old label, old label) to (new label, new label); the edge is
//             counted by its source when the source moved, else by its target.
//             (The per-vertex change vectors used for scoring cannot simply be
//             added up: two adjacent vertices that move together change their
//             shared edge's entry once, not twice.)  Workgroup deltas of M in
//             LDS are flushed with integer atomics, so M does not depend on
//             thread order;
//   apply  -- M += delta, labels of accepted vertices;
//   final  -- block degrees, proposal tables, DL (one workgroup, fixed order).
#include <string.h>

#include "sbp_internal.h"

namespace sbp {

namespace {

constexpr int DC = SBP_DENSE_MAX_C_DEV;
constexpr int FTAB_N = SBP_FTAB_N;

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

// f(x) = x ln x for every integer 0 <= x < FTAB_N, computed on the device with
// the same xlogx as the direct evaluation, so a lookup returns the very value
// a direct evaluation would.
__global__ void k_ftab(double *__restrict__ tab) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < FTAB_N; i += gridDim.x * blockDim.x)
        tab[i] = xlogx((double)i);
}
__device__ __forceinline__ double fx(const double *__restrict__ tab, int x) {
    return x < FTAB_N ? tab[x] : xlogx((double)x);
}

// Degrees, proposal tables and DL from M; sweep totals (one workgroup of 1024).
__global__ void __launch_bounds__(1024) k_dense_final(GDev g, DenseBM bm, const long long *__restrict__ stats_part,
                                                      const double *__restrict__ sum_part, int nwg,
                                                      sbp_sweep_stats_dev *__restrict__ stats) {
    __shared__ int Ms[DC * DC];
    __shared__ int so[DC], si[DC];
    __shared__ double wred[16];
    __shared__ long long lred[3][16];
    __shared__ double sred[16];
    const int C = g.C, CC = C * C, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const double *tab = bm.ftab;
    for (int i = tid; i < CC; i += 1024) Ms[i] = bm.M[i];
    __syncthreads();
    if (tid < C) {
        int x = 0, run = 0;
        for (int b = 0; b < C; ++b) {
            x += Ms[tid * C + b];
            run += Ms[tid * C + b] + Ms[b * C + tid];
            bm.cdf[tid * C + b] = run;
        }
        so[tid] = x;
        bm.dout[tid] = x;
    } else if (tid >= 64 && tid < 64 + C) {
        const int t = tid - 64;
        int x = 0;
        for (int a = 0; a < C; ++a) x += Ms[a * C + t];
        si[t] = x;
        bm.din[t] = x;
    }
    __syncthreads();
    // L = sum f(M) - sum f(dout) - sum f(din), fixed order
    double acc = 0.0;
    for (int i = tid; i < CC; i += 1024) acc += fx(tab, Ms[i]);
    if (tid < C) acc -= fx(tab, so[tid]);
    else if (tid >= 64 && tid < 64 + C) acc -= fx(tab, si[tid - 64]);
    acc = wave_sum(acc);
    long long a0 = 0, a1 = 0, a2 = 0;
    double sd = 0.0;
    if (stats)
        for (int w = tid; w < nwg; w += 1024) {
            a0 += stats_part[4 * w + 0];
            a1 += stats_part[4 * w + 1];
            a2 += stats_part[4 * w + 2];
            sd += sum_part[w];
        }
    a0 = wave_sum_i64(a0);
    a1 = wave_sum_i64(a1);
    a2 = wave_sum_i64(a2);
    sd = wave_sum(sd);
    if (lane == 0) {
        wred[wv] = acc;
        lred[0][wv] = a0;
        lred[1][wv] = a1;
        lred[2][wv] = a2;
        sred[wv] = sd;
    }
    __syncthreads();
    if (tid == 0) {
        double L = 0.0, sdt = 0.0;
        long long p = 0, sp = 0, ac = 0;
        for (int w = 0; w < 16; ++w) {
            L += wred[w];
            p += lred[0][w];
            sp += lred[1][w];
            ac += lred[2][w];
            sdt += sred[w];
        }
        const double dl = model_terms_d((double)g.e, (double)g.n, (double)C) - L;
        bm.dl[0] = dl;
        if (stats) {
            stats->proposals += p;
            stats->self_proposals += sp;
            stats->accepted += ac;
            stats->sum_dS_accepted += sdt;
            stats->dl_after = dl;
        }
    }
}

template <int GS>
__device__ __forceinline__ double group_sum(double x) {
#pragma unroll
    for (int o = GS / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, SBP_WAVE);
    return x;
}

constexpr int CH = 64;     // vertices per chunk
constexpr int EVAL_T = 256;  // threads per workgroup
constexpr int GS = 16;     // lanes per vertex in the scoring phase
constexpr int UA = 4;      // edge ends in flight per thread in the gather phase

// Byte offsets of the evaluation kernel's dynamic LDS for C blocks.
struct EvalOff {
    int fdo, fdi, inv, W, wst, wsd, Ms, cdf, dsum, dos, dis, H, v, r, op, kout, ip, kin, pre, ell, t0, j0, bytes;
};
__host__ __device__ __forceinline__ int al8(int x) { return (x + 7) & ~7; }
__host__ __device__ __forceinline__ EvalOff eval_offsets(int C) {
    EvalOff o;
    int p = 0;
    o.fdo = p; p += 8 * C;
    o.fdi = p; p += 8 * C;
    o.inv = p; p += 8 * C;
    o.W = p; p += 8 * 4 * CH;
    o.wst = p; p += 8 * 3 * (EVAL_T / 64);
    o.wsd = p; p += 8 * (EVAL_T / 64);
    o.Ms = p; p += 4 * C * C;
    o.cdf = p; p += 4 * C * C;
    o.dsum = p; p += 4 * C;
    o.dos = p; p += 4 * C;
    o.dis = p; p += 4 * C;
    o.H = p; p += 4 * CH * C;
    o.v = p; p += 4 * CH;
    o.r = p; p += 4 * CH;
    o.op = p; p += 4 * CH;
    o.kout = p; p += 4 * CH;
    o.ip = p; p += 4 * CH;
    o.kin = p; p += 4 * CH;
    o.pre = p; p += 4 * (CH + 1);
    o.ell = p; p += 4 * CH;
    o.t0 = p; p += 4 * CH;
    o.j0 = p; p += 4 * CH;
    o.bytes = al8(p);
    return o;
}

// Sweep batch evaluation against the snapshot M.  A workgroup takes CH batch
// vertices at a time: (0) their pointers, labels and Philox words; (A) every
// edge end of the chunk in one flattened, balanced loop (coalesced ids, label
// gathers all in flight) into packed per-vertex block histograms in LDS;
// (B) groups of GS lanes score GS vertices per round from LDS, lane l of a
// group owning blocks t = l, l + GS, ...
__global__ void __launch_bounds__(EVAL_T, 4) k_dense_eval(GDev g, DenseBM bm, int *__restrict__ nb, SweepTraceDev tr,
                                                      long long *__restrict__ stats_part, double *__restrict__ sum_part) {
    extern __shared__ __align__(16) char smem[];
    const EvalOff o = eval_offsets(g.C);
    struct {
        double *fdo, *fdi, *inv;
        uint64_t *W;
        long long *wst;
        double *wsd;
        int *Ms, *cdf, *dsum, *dos, *dis;
        unsigned *H;
        int *v, *r, *op, *kout, *ip, *kin, *pre, *ell, *t0, *j0;
    } L = {(double *)(smem + o.fdo), (double *)(smem + o.fdi), (double *)(smem + o.inv),
           (uint64_t *)(smem + o.W), (long long *)(smem + o.wst), (double *)(smem + o.wsd),
           (int *)(smem + o.Ms), (int *)(smem + o.cdf), (int *)(smem + o.dsum), (int *)(smem + o.dos),
           (int *)(smem + o.dis), (unsigned *)(smem + o.H), (int *)(smem + o.v), (int *)(smem + o.r),
           (int *)(smem + o.op), (int *)(smem + o.kout), (int *)(smem + o.ip), (int *)(smem + o.kin),
           (int *)(smem + o.pre), (int *)(smem + o.ell), (int *)(smem + o.t0), (int *)(smem + o.j0)};
    const double *__restrict__ tab = bm.ftab;
    const int C = g.C, CC = C * C;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int grp = tid / GS, gl = tid % GS, wgrp = lane / GS;  // group in workgroup / in wave
    const double eps = (double)g.eps, epsC = (double)g.eps * (double)C;
    const long long eC = (long long)g.eps * C;
    for (int i = tid; i < CC; i += EVAL_T) {
        L.Ms[i] = bm.M[i];
        L.cdf[i] = bm.cdf[i];
    }
    if (tid < C) {
        const int o = bm.dout[tid], n = bm.din[tid];
        L.dos[tid] = o;
        L.dis[tid] = n;
        L.dsum[tid] = o + n;
        L.fdo[tid] = fx(tab, o);
        L.fdi[tid] = fx(tab, n);
        L.inv[tid] = 1.0 / ((double)(o + n) + epsC);
    }
    long long n_prop = 0, n_self = 0, n_acc = 0;
    double s_dS = 0.0;
    const int nbc = (g.n - g.batch + g.n_batches - 1) / g.n_batches;
    const int nchunks = (nbc + CH - 1) / CH;
    const uint32_t k0 = (uint32_t)g.seed, k1 = (uint32_t)(g.seed >> 32);
    for (int chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
        __syncthreads();  // previous chunk done with the LDS
        const int base = chunk * CH;
        const int nv = min(CH, nbc - base);
        // (0) vertex data and words
        if (tid < CH) {
            int k = 0;
            if (tid < nv) {
                const int v = g.batch + (base + tid) * g.n_batches;
                const int op = g.out_ptr[v], ko = g.out_ptr[v + 1] - op;
                const int ip = g.in_ptr[v], ki = g.in_ptr[v + 1] - ip;
                L.v[tid] = v;
                L.r[tid] = g.lab[v];
                L.op[tid] = op;
                L.kout[tid] = ko;
                L.ip[tid] = ip;
                L.kin[tid] = ki;
                k = ko + ki;
                uint32_t wa[4], wb[4];
                philox_block((uint32_t)v, g.sweep, 0u, 0u, k0, k1, wa);
                philox_block((uint32_t)v, g.sweep, 1u, 0u, k0, k1, wb);
                const uint64_t W0 = (uint64_t)wa[0] | ((uint64_t)wa[1] << 32);
                L.W[4 * tid + 0] = W0;
                L.W[4 * tid + 1] = (uint64_t)wa[2] | ((uint64_t)wa[3] << 32);
                L.W[4 * tid + 2] = (uint64_t)wb[0] | ((uint64_t)wb[1] << 32);
                L.W[4 * tid + 3] = (uint64_t)wb[2] | ((uint64_t)wb[3] << 32);
                L.j0[tid] = k > 0 ? (int)draw_idx(W0, (uint64_t)k) : -1;
            }
            L.ell[tid] = 0;
            // exclusive prefix of the edge-end counts (wave 0)
            int x = k;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o, SBP_WAVE);
                if (lane >= o) x += y;
            }
            L.pre[tid + 1] = x;
            if (tid == 0) L.pre[0] = 0;
        }
        for (int i = tid; i < CH * C; i += EVAL_T) L.H[i] = 0;
        __syncthreads();
        // (A) all edge ends of the chunk, UA at a time per thread with every
        // load issued before its use
        const int total = L.pre[nv];
        for (int f0 = tid; f0 < total; f0 += EVAL_T * UA) {
            int vi[UA], j[UA], u[UA];
#pragma unroll
            for (int q = 0; q < UA; ++q) {
                const int f = f0 + q * EVAL_T;
                int lo = 0, hi = nv - 1;  // last vertex with pre <= f
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (L.pre[mid] <= f) lo = mid; else hi = mid - 1;
                }
                vi[q] = f < total ? lo : -1;
                j[q] = f - L.pre[lo];
            }
#pragma unroll
            for (int q = 0; q < UA; ++q) {
                u[q] = -1;
                if (vi[q] >= 0) {
                    const int ko = L.kout[vi[q]];
                    u[q] = j[q] < ko ? g.out_idx[L.op[vi[q]] + j[q]] : g.in_idx[L.ip[vi[q]] + (j[q] - ko)];
                }
            }
            int t[UA];
#pragma unroll
            for (int q = 0; q < UA; ++q) t[q] = (vi[q] >= 0 && u[q] != L.v[vi[q]]) ? g.lab[u[q]] : -1;
#pragma unroll
            for (int q = 0; q < UA; ++q) {
                if (vi[q] < 0) continue;
                const bool out = j[q] < L.kout[vi[q]];
                int tt = t[q];
                if (tt < 0) {  // self-loop end
                    tt = L.r[vi[q]];
                    if (out) atomicAdd(&L.ell[vi[q]], 1);
                } else {
                    atomicAdd(&L.H[vi[q] * C + tt], out ? 1u : 65536u);
                }
                if (j[q] == L.j0[vi[q]]) L.t0[vi[q]] = tt;
            }
        }
        __syncthreads();
        // (B) scoring, GS vertices per round (64/GS per wave)
        for (int vi = grp; vi < CH; vi += EVAL_T / GS) {
            const bool valid = vi < nv;
            int v = 0, r = 0, kout = 0, kin = 0, ell = 0;
            uint64_t W1 = 0, W2 = 0, W3 = 0;
            if (valid) {
                v = L.v[vi];
                r = L.r[vi];
                kout = L.kout[vi];
                kin = L.kin[vi];
                ell = L.ell[vi];
                W1 = L.W[4 * vi + 1];
                W2 = L.W[4 * vi + 2];
                W3 = L.W[4 * vi + 3];
            }
            const int k = kout + kin;
            const unsigned *Hv = L.H + vi * C;
            int s;
            if (k == 0) {
                s = (int)draw_idx(W2, (uint64_t)C);
            } else {
                const int t0 = L.t0[vi];
                const long long dt = L.dsum[t0];
                if (draw_idx(W1, (uint64_t)(dt + eC)) < eC) {
                    s = (int)draw_idx(W2, (uint64_t)C);
                } else {
                    const long long x = draw_idx(W2, (uint64_t)dt);
                    s = C;
                    for (int b0 = 0; b0 < C; b0 += GS) {
                        const int cand = b0 + gl;
                        const bool hit = cand < C && (long long)L.cdf[t0 * C + cand] > x;
                        const uint64_t m = (__ballot(hit) >> (wgrp * GS)) & ((1ull << GS) - 1);
                        if (m && s == C) s = b0 + __builtin_ctzll(m);
                    }
                }
            }
            const bool act = valid && s != r;
            if (!act) s = r;  // keeps every index below in range
            const int *Ms = L.Ms;
            double dL = 0.0, qf = 0.0, qr = 0.0;
            // blocks t != r, s: changed entries of rows r, s and columns r, s
#pragma unroll 2
            for (int t = gl; t < C; t += GS) {
                const unsigned h = (act && t != r && t != s) ? Hv[t] : 0u;
                if (h) {
                    const int ko = (int)(h & 0xffffu), ki = (int)(h >> 16);
                    const int rt = r * C + t, st = s * C + t, tr_ = t * C + r, ts = t * C + s;
                    const int Mrt = Ms[rt], Mst = Ms[st], Mtr = Ms[tr_], Mts = Ms[ts];
                    // a zero count contributes exactly zero
                    dL += fx(tab, Mrt - ko) - fx(tab, Mrt) + fx(tab, Mst + ko) - fx(tab, Mst);
                    dL += fx(tab, Mtr - ki) - fx(tab, Mtr) + fx(tab, Mts + ki) - fx(tab, Mts);
                    const double kt = (double)(ko + ki);
                    qf += kt * (((double)(Mts + Mst) + eps) * L.inv[t]);
                    qr += kt * (((double)(Mtr - ki + Mrt - ko) + eps) * L.inv[t]);
                }
            }
            // the 2x2 corner (r, s) x (r, s), the four block degrees and the
            // Hastings terms of t = r and t = s: one item per lane, branch-free
            {
                const unsigned hr = Hv[r], hs = Hv[s];
                const int ko_r = (int)(hr & 0xffffu), ki_r = (int)(hr >> 16);
                const int ko_s = (int)(hs & 0xffffu), ki_s = (int)(hs >> 16);
                const int Mrr = Ms[r * C + r], Mrs = Ms[r * C + s], Msr = Ms[s * C + r], Mss = Ms[s * C + s];
                const int drr = -ko_r - ki_r - ell, drs = -ko_s + ki_r, dsr = ko_r - ki_s, dss = ko_s + ki_s + ell;
                const int c = gl & 3;
                // entries (lanes 0-3) and degrees (lanes 4-7)
                const int m_old = c == 0 ? Mrr : c == 1 ? Mrs : c == 2 ? Msr : Mss;
                const int m_d = c == 0 ? drr : c == 1 ? drs : c == 2 ? dsr : dss;
                const int deg_old = c == 0 ? L.dos[r] : c == 1 ? L.dos[s] : c == 2 ? L.dis[r] : L.dis[s];
                const int deg_d = c == 0 ? -kout : c == 1 ? kout : c == 2 ? -kin : kin;
                const bool is_m = gl < 4;
                const int old = is_m ? m_old : deg_old, nw = old + (is_m ? m_d : deg_d);
                if (act && gl < 8) dL += (is_m ? 1.0 : -1.0) * (fx(tab, nw) - fx(tab, old));
                // Hastings terms (lanes 8-11): t = r and t = s before, t = r and t = s after
                const int kk = c == 0 ? ko_r + ki_r + 2 * ell : c == 1 ? ko_s + ki_s : c == 2 ? ko_r + ki_r : ko_s + ki_s + 2 * ell;
                const int num = c == 0 ? Mrs + Msr : c == 1 ? 2 * Mss : c == 2 ? 2 * (Mrr + drr) : Msr + dsr + Mrs + drs;
                const int den = c == 0 ? L.dsum[r] : c == 1 ? L.dsum[s] : c == 2 ? L.dsum[r] - k : L.dsum[s] + k;
                if (act && gl >= 8 && gl < 12 && kk) {
                    const double term = (double)kk * (((double)num + eps) / ((double)den + epsC));
                    if (c < 2) qf += term; else qr += term;
                }
            }
            dL = group_sum<GS>(dL);
            qf = group_sum<GS>(qf);
            qr = group_sum<GS>(qr);
            // the three logs of the wave's 64/GS vertices in one evaluation
            double lg;
            {
                const double u = draw_unit(W3);
                const int q = lane / 3, m = lane % 3;
                const int src = (q < 64 / GS ? q : 0) * GS;
                const double xr = __shfl(qr, src, SBP_WAVE), xf = __shfl(qf, src, SBP_WAVE);
                const double xu = __shfl(u, src, SBP_WAVE);
                double arg = m == 0 ? xr : m == 1 ? xf : xu;
                if (!(arg > 0.0)) arg = 1.0;
                lg = log(arg);
            }
            const double lnqr = __shfl(lg, 3 * wgrp + 0, SBP_WAVE);
            const double lnqf = __shfl(lg, 3 * wgrp + 1, SBP_WAVE);
            const double lnu = __shfl(lg, 3 * wgrp + 2, SBP_WAVE);
            const double dS = -dL;
            const double lnH = (act && k > 0) ? lnqr - lnqf : 0.0;
            const double z = -g.beta * dS + lnH;
            const bool acc = act && lnu < z;
            if (gl == 0 && valid) {
                ++n_prop;
                if (!act) ++n_self;
                if (acc) {
                    ++n_acc;
                    s_dS += dS;
                }
                const int uu = g.voff + v;
                nb[v] = acc ? s : -1;
                if (tr.prop) tr.prop[uu] = act ? s : r;
                if (tr.dS) tr.dS[uu] = act ? dS : 0.0;
                if (tr.lnH) tr.lnH[uu] = act ? lnH : 0.0;
                if (tr.margin) tr.margin[uu] = act ? z - lnu : 0.0;
                if (tr.accept) tr.accept[uu] = acc ? 1 : 0;
                if (tr.status) tr.status[uu] = act ? (acc ? 1 : 0) : -1;
            }
        }
    }
    n_prop = wave_sum_i64(n_prop);
    n_self = wave_sum_i64(n_self);
    n_acc = wave_sum_i64(n_acc);
    s_dS = wave_sum(s_dS);
    __syncthreads();
    if (lane == 0) {
        L.wst[3 * wv + 0] = n_prop;
        L.wst[3 * wv + 1] = n_self;
        L.wst[3 * wv + 2] = n_acc;
        L.wsd[wv] = s_dS;
    }
    __syncthreads();
    if (tid == 0) {
        long long a = 0, b2 = 0, c = 0;
        double sd = 0.0;
        for (int w = 0; w < EVAL_T / 64; ++w) {
            a += L.wst[3 * w + 0];
            b2 += L.wst[3 * w + 1];
            c += L.wst[3 * w + 2];
            sd += L.wsd[w];
        }
        stats_part[4 * blockIdx.x + 0] = a;
        stats_part[4 * blockIdx.x + 1] = b2;
        stats_part[4 * blockIdx.x + 2] = c;
        stats_part[4 * blockIdx.x + 3] = 0;
        sum_part[blockIdx.x] = sd;
    }
}

// Change of M from the moves of a single-batch sweep, edge-parallel: every
// out-edge (u, w) whose endpoints' labels changed moves one count from
// (old u, old w) to (new u, new w).  Chunks of CH vertices per workgroup.
__global__ void __launch_bounds__(EVAL_T) k_dense_delta_edges(GDev g, const int *__restrict__ nb,
                                                             int *__restrict__ delta) {
    extern __shared__ __align__(16) char smem[];
    const int C = g.C, CC = C * C, tid = threadIdx.x, lane = tid & 63;
    int *dl = (int *)smem;
    int *pre = dl + CC;        // [CH+1]
    int *op = pre + CH + 1;    // [CH]
    int *a0 = op + CH;         // old label of the chunk vertex
    int *a1 = a0 + CH;         // new label
    for (int i = tid; i < CC; i += EVAL_T) dl[i] = 0;
    const int nchunks = (g.n + CH - 1) / CH;
    for (int chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
        __syncthreads();
        const int base = chunk * CH, nv = min(CH, g.n - base);
        if (tid < CH) {
            int k = 0;
            if (tid < nv) {
                const int v = base + tid;
                const int o = g.out_ptr[v];
                k = g.out_ptr[v + 1] - o;
                op[tid] = o;
                const int old = g.lab[v], x = nb[v];
                a0[tid] = old;
                a1[tid] = x >= 0 ? x : old;
            }
            int x = k;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o, SBP_WAVE);
                if (lane >= o) x += y;
            }
            pre[tid + 1] = x;
            if (tid == 0) pre[0] = 0;
        }
        __syncthreads();
        const int total = pre[nv];
        for (int f0 = tid; f0 < total; f0 += EVAL_T * UA) {
            int vi[UA], w[UA];
#pragma unroll
            for (int q = 0; q < UA; ++q) {
                const int f = f0 + q * EVAL_T;
                int lo = 0, hi = nv - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (pre[mid] <= f) lo = mid; else hi = mid - 1;
                }
                vi[q] = f < total ? lo : -1;
                w[q] = vi[q] >= 0 ? g.out_idx[op[lo] + (f - pre[lo])] : 0;
            }
            int b[UA], xw[UA];
#pragma unroll
            for (int q = 0; q < UA; ++q) {
                b[q] = vi[q] >= 0 ? g.lab[w[q]] : 0;
                xw[q] = vi[q] >= 0 ? nb[w[q]] : -1;
            }
#pragma unroll
            for (int q = 0; q < UA; ++q) {
                if (vi[q] < 0) continue;
                const int b2 = xw[q] >= 0 ? xw[q] : b[q];
                const int a = a0[vi[q]], a2 = a1[vi[q]];
                if (a != a2 || b[q] != b2) {
                    atomicAdd(&dl[a * C + b[q]], -1);
                    atomicAdd(&dl[a2 * C + b2], 1);
                }
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < CC; i += EVAL_T)
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

// M += delta (delta cleared for the next batch); labels of accepted moves.
__global__ void k_dense_apply(GDev g, DenseBM bm, int *__restrict__ delta, const int *__restrict__ nb) {
    const int CC = g.C * g.C;
    const int nbc = (g.n - g.batch + g.n_batches - 1) / g.n_batches;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < CC + nbc; i += gridDim.x * blockDim.x) {
        if (i < CC) {
            const int x = delta[i];
            if (x) {
                bm.M[i] += x;
                delta[i] = 0;
            }
        } else {
            const int v = g.batch + (i - CC) * g.n_batches;
            const int x = nb[v];
            if (x >= 0) g.lab[v] = x;
        }
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
            const int t = __builtin_ctzll(__ballot(lane < C && (long long)bm.cdf[c * C + lane] > x0));
            const long long dt = (long long)bm.dout[t] + bm.din[t];
            if (draw_idx(W.w[1], (uint64_t)(dt + eC)) < eC) {
                const int kk = (int)draw_idx(W.w[2], (uint64_t)(C - 1));
                cp = kk + (kk >= c);
            } else {
                const long long x2 = draw_idx(W.w[2], (uint64_t)dt);
                cp = __builtin_ctzll(__ballot(lane < C && (long long)bm.cdf[t * C + lane] > x2));
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

int dense_build(const GDev &g, DenseBM &bm, int *delta, hipStream_t s) {
    const int CC = g.C * g.C;
    hipLaunchKernelGGL(k_zero, dim3(grid_for(CC, 256, 64)), dim3(256), 0, s, bm.M, CC);
    hipLaunchKernelGGL(k_zero, dim3(grid_for(CC, 256, 64)), dim3(256), 0, s, delta, CC);
    hipLaunchKernelGGL(k_ftab, dim3(FTAB_N / 256), dim3(256), 0, s, bm.ftab);
    hipLaunchKernelGGL(k_dense_hist, dim3(grid_for(g.n, 256, 1024)), dim3(256), 0, s, g, bm.M);
    hipLaunchKernelGGL(k_dense_final, dim3(1), dim3(1024), 0, s, g, bm, (const long long *)nullptr,
                       (const double *)nullptr, 0, (sbp_sweep_stats_dev *)nullptr);
    SBP_LAUNCH_CHECK();
    return 0;
}

int g_eval_wgs = 0;     // workgroups of the evaluation grid (0 = one per chunk, capped by ws.nwg)
int g_delta_wgs = 1024;  // workgroups of the edge-parallel delta grid

int dense_sweep_batch(const GDev &g, DenseBM &bm, DenseScratch &ws, const SweepTraceDev &tr,
                      sbp_sweep_stats_dev *stats, hipStream_t s) {
    const int nbc = (g.n - g.batch + g.n_batches - 1) / g.n_batches;
    const int nchunks = (nbc + CH - 1) / CH;
    int grid = nchunks < ws.nwg ? nchunks : ws.nwg;
    if (g_eval_wgs > 0 && grid > g_eval_wgs) grid = g_eval_wgs;
    if (grid < 1) grid = 1;
    const size_t lds = (size_t)eval_offsets(g.C).bytes;
    {
        ProfileScope prof("sweep_eval", s);
        hipLaunchKernelGGL(k_dense_eval, dim3(grid), dim3(EVAL_T), lds, s, g, bm, ws.nb, tr, ws.stats_part,
                           ws.sum_part);
    }
    if (g.n_batches == 1) {
        const size_t dl_lds = sizeof(int) * ((size_t)g.C * g.C + 4 * CH + 1);
        int dgrid = (g.n + CH - 1) / CH;
        if (dgrid > g_delta_wgs) dgrid = g_delta_wgs;
        hipLaunchKernelGGL(k_dense_delta_edges, dim3(dgrid), dim3(EVAL_T), dl_lds, s, g, (const int *)ws.nb, ws.delta);
    } else {
        hipLaunchKernelGGL(k_dense_delta, dim3(grid), dim3(256), 0, s, g, (const int *)ws.nb, ws.delta);
    }
    hipLaunchKernelGGL(k_dense_apply, dim3(grid_for(g.C * g.C + nbc, 256, 2048)), dim3(256), 0, s, g, bm, ws.delta,
                       ws.nb);
    hipLaunchKernelGGL(k_dense_final, dim3(1), dim3(1024), 0, s, g, bm, ws.stats_part, ws.sum_part, grid, stats);
    SBP_LAUNCH_CHECK();
    return 0;
}

int dense_tune(const char *key, long long value) {
    if (!strcmp(key, "dense_eval_workgroups") && value >= 0) {
        g_eval_wgs = (int)value;
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

}  // namespace sbp
