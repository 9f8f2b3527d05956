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
#include "sbp_internal.h"

namespace sbp {

namespace {

constexpr int DC = SBP_DENSE_MAX_C_DEV;
constexpr int EVAL_WAVES = 4;

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

// Degrees, proposal tables and DL from M (one workgroup of 1024 threads).
__global__ void __launch_bounds__(1024) k_dense_final(GDev g, DenseBM bm, const long long *__restrict__ stats_part,
                                                      const double *__restrict__ sum_part, int nwg,
                                                      sbp_sweep_stats_dev *__restrict__ stats) {
    __shared__ int Ms[DC * DC];
    __shared__ double wred[16];
    const int C = g.C, CC = C * C, tid = threadIdx.x;
    for (int i = tid; i < CC; i += 1024) Ms[i] = bm.M[i];
    __syncthreads();
    if (tid < C) {
        int so = 0, si = 0;
        for (int b = 0; b < C; ++b) {
            so += Ms[tid * C + b];
            si += Ms[b * C + tid];
        }
        bm.dout[tid] = so;
        bm.din[tid] = si;
        int run = 0;
        for (int s = 0; s < C; ++s) {
            run += Ms[tid * C + s] + Ms[s * C + tid];
            bm.cdf[tid * C + s] = run;
        }
    }
    // L = sum f(M) - sum f(dout) - sum f(din)
    double acc = 0.0;
    for (int i = tid; i < CC; i += 1024) acc += xlogx((double)Ms[i]);
    if (tid < C) {
        int so = 0, si = 0;
        for (int b = 0; b < C; ++b) {
            so += Ms[tid * C + b];
            si += Ms[b * C + tid];
        }
        acc -= xlogx((double)so) + xlogx((double)si);
    }
    acc = wave_sum(acc);
    if ((tid & 63) == 0) wred[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double L = 0.0;
        for (int w = 0; w < 16; ++w) L += wred[w];
        const double dl = model_terms_d((double)g.e, (double)g.n, (double)C) - L;
        bm.dl[0] = dl;
        if (stats) {
            long long p = 0, sp = 0, a = 0;
            double sd = 0.0;
            for (int w = 0; w < nwg; ++w) {
                p += stats_part[4 * w + 0];
                sp += stats_part[4 * w + 1];
                a += stats_part[4 * w + 2];
                sd += sum_part[w];
            }
            stats->proposals += p;
            stats->self_proposals += sp;
            stats->accepted += a;
            stats->sum_dS_accepted += sd;
            stats->dl_after = dl;
        }
    }
}

// Sweep batch evaluation, wave per vertex, lane t <-> block t.
__global__ void __launch_bounds__(EVAL_WAVES * 64) k_dense_eval(GDev g, DenseBM bm, int *__restrict__ nb,
                                                               SweepTraceDev tr,
                                                               long long *__restrict__ stats_part,
                                                               double *__restrict__ sum_part) {
    __shared__ int Ms[DC * DC];
    __shared__ int dsum[DC];          // d_t = d_t^out + d_t^in
    __shared__ int dos[DC], dis[DC];
    __shared__ int hist[EVAL_WAVES][2][DC];
    __shared__ long long wst[EVAL_WAVES][3];
    __shared__ double wsd[EVAL_WAVES];
    const int C = g.C, CC = C * C;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int i = tid; i < CC; i += blockDim.x) Ms[i] = bm.M[i];
    if (tid < C) {
        dos[tid] = bm.dout[tid];
        dis[tid] = bm.din[tid];
        dsum[tid] = bm.dout[tid] + bm.din[tid];
    }
    __syncthreads();
    const double eps = (double)g.eps, epsC = (double)g.eps * (double)C;
    const long long eC = (long long)g.eps * C;
    long long n_prop = 0, n_self = 0, n_acc = 0;
    double s_dS = 0.0;
    const int nb_count = (g.n - g.batch + g.n_batches - 1) / g.n_batches;
    const int gw = blockIdx.x * EVAL_WAVES + wv, nw = gridDim.x * EVAL_WAVES;
    int *hout = hist[wv][0], *hin = hist[wv][1];
    for (int idx = gw; idx < nb_count; idx += nw) {
        const int v = g.batch + idx * g.n_batches;
        const int r = g.lab[v];
        const int op = g.out_ptr[v], kout = g.out_ptr[v + 1] - op;
        const int ip = g.in_ptr[v], kin = g.in_ptr[v + 1] - ip;
        const int k = kout + kin;
        hout[lane] = 0;
        hin[lane] = 0;
        wave_sync_lds();
        int ell = 0;
        for (int j = lane; j < k; j += 64) {
            const int u = j < kout ? g.out_idx[op + j] : g.in_idx[ip + j - kout];
            if (u == v) {
                if (j < kout) ++ell;
            } else {
                atomicAdd(j < kout ? &hout[g.lab[u]] : &hin[g.lab[u]], 1);
            }
        }
        ell = wave_sum_i32(ell);
        wave_sync_lds();
        const int ko = lane < C ? hout[lane] : 0, ki = lane < C ? hin[lane] : 0;
        const Words4 W = draw_words(g.seed, (uint32_t)v, g.sweep, 0u, 0u);
        int s;
        if (k == 0) {
            s = (int)draw_idx(W.w[2], (uint64_t)C);
        } else {
            const int j0 = (int)draw_idx(W.w[0], (uint64_t)k);
            const int u0 = j0 < kout ? g.out_idx[op + j0] : g.in_idx[ip + j0 - kout];
            const int t0 = g.lab[u0];
            const long long dt = dsum[t0];
            if (draw_idx(W.w[1], (uint64_t)(dt + eC)) < eC) {
                s = (int)draw_idx(W.w[2], (uint64_t)C);
            } else {
                const long long x = draw_idx(W.w[2], (uint64_t)dt);
                const uint64_t hit = __ballot(lane < C && (long long)bm.cdf[t0 * C + lane] > x);
                s = __builtin_ctzll(hit);
            }
        }
        const double lnu = log(draw_unit(W.w[3]));
        ++n_prop;
        const int u = g.voff + v;
        if (s == r) {
            ++n_self;
            if (lane == 0) {
                nb[v] = -1;
                if (tr.prop) tr.prop[u] = s;
                if (tr.dS) tr.dS[u] = 0.0;
                if (tr.lnH) tr.lnH[u] = 0.0;
                if (tr.margin) tr.margin[u] = 0.0;
                if (tr.accept) tr.accept[u] = 0;
                if (tr.status) tr.status[u] = -1;
            }
            continue;
        }
        double dL = 0.0, qf = 0.0, qr = 0.0;
        const int t = lane;
        if (t < C && t != r && t != s) {
            const int Mrt = Ms[r * C + t], Mst = Ms[s * C + t], Mtr = Ms[t * C + r], Mts = Ms[t * C + s];
            if (ko) dL += xlogx((double)(Mrt - ko)) - xlogx((double)Mrt) + xlogx((double)(Mst + ko)) - xlogx((double)Mst);
            if (ki) dL += xlogx((double)(Mtr - ki)) - xlogx((double)Mtr) + xlogx((double)(Mts + ki)) - xlogx((double)Mts);
            if (ko + ki) {
                const double kt = (double)(ko + ki);
                const double den = (double)dsum[t] + epsC;
                qf += kt * (((double)(Mts + Mst) + eps) / den);
                qr += kt * (((double)(Mtr - ki + Mrt - ko) + eps) / den);
            }
        }
        const int ko_r = __shfl(ko, r, SBP_WAVE), ki_r = __shfl(ki, r, SBP_WAVE);
        const int ko_s = __shfl(ko, s, SBP_WAVE), ki_s = __shfl(ki, s, SBP_WAVE);
        if (lane == 0) {
            const int Mrr = Ms[r * C + r], Mrs = Ms[r * C + s], Msr = Ms[s * C + r], Mss = Ms[s * C + s];
            const int drr = -ko_r - ki_r - ell, drs = -ko_s + ki_r, dsr = ko_r - ki_s, dss = ko_s + ki_s + ell;
            dL += xlogx((double)(Mrr + drr)) - xlogx((double)Mrr);
            dL += xlogx((double)(Mrs + drs)) - xlogx((double)Mrs);
            dL += xlogx((double)(Msr + dsr)) - xlogx((double)Msr);
            dL += xlogx((double)(Mss + dss)) - xlogx((double)Mss);
            const double dor = dos[r], dosv = dos[s], dir = dis[r], disv = dis[s];
            dL -= xlogx(dor - kout) - xlogx(dor) + xlogx(dosv + kout) - xlogx(dosv);
            dL -= xlogx(dir - kin) - xlogx(dir) + xlogx(disv + kin) - xlogx(disv);
            const double kd = (double)k;
            const double d_r = dor + dir, d_s = dosv + disv;
            const int kr = ko_r + ki_r + 2 * ell, ks = ko_s + ki_s;
            if (kr) qf += (double)kr * (((double)(Mrs + Msr) + eps) / (d_r + epsC));
            if (ks) qf += (double)ks * (((double)(2 * Mss) + eps) / (d_s + epsC));
            const int kr2 = ko_r + ki_r, ks2 = ko_s + ki_s + 2 * ell;
            if (kr2) qr += (double)kr2 * (((double)(2 * (Mrr + drr)) + eps) / (d_r - kd + epsC));
            if (ks2) qr += (double)ks2 * (((double)(Msr + dsr + Mrs + drs) + eps) / (d_s + kd + epsC));
        }
        dL = wave_sum(dL);
        qf = wave_sum(qf);
        qr = wave_sum(qr);
        const double dS = -dL;
        const double lnH = k > 0 ? log(qr) - log(qf) : 0.0;
        const double z = -g.beta * dS + lnH;
        const bool acc = lnu < z;
        if (acc) {
            ++n_acc;
            s_dS += dS;
        }
        if (lane == 0) {
            nb[v] = acc ? s : -1;
            if (tr.prop) tr.prop[u] = s;
            if (tr.dS) tr.dS[u] = dS;
            if (tr.lnH) tr.lnH[u] = lnH;
            if (tr.margin) tr.margin[u] = z - lnu;
            if (tr.accept) tr.accept[u] = acc ? 1 : 0;
            if (tr.status) tr.status[u] = acc ? 1 : 0;
        }
    }
    if (lane == 0) {
        wst[wv][0] = n_prop;
        wst[wv][1] = n_self;
        wst[wv][2] = n_acc;
        wsd[wv] = s_dS;
    }
    __syncthreads();
    if (tid == 0) {
        long long a = 0, b = 0, c = 0;
        double sd = 0.0;
        for (int w = 0; w < EVAL_WAVES; ++w) {
            a += wst[w][0];
            b += wst[w][1];
            c += wst[w][2];
            sd += wsd[w];
        }
        stats_part[4 * blockIdx.x + 0] = a;
        stats_part[4 * blockIdx.x + 1] = b;
        stats_part[4 * blockIdx.x + 2] = c;
        stats_part[4 * blockIdx.x + 3] = 0;
        sum_part[blockIdx.x] = sd;
    }
}

// Change of M from the accepted moves of one batch, exact for moves of
// adjacent vertices: edge (u, w) goes from (old u, old w) to (new u, new w).
__global__ void __launch_bounds__(256) k_dense_delta(GDev g, const int *__restrict__ nb, int *__restrict__ delta) {
    __shared__ int dl[DC * DC];
    const int C = g.C, CC = C * C;
    const int tid = threadIdx.x, lane = tid & 63;
    for (int i = tid; i < CC; i += blockDim.x) dl[i] = 0;
    __syncthreads();
    const int nbc = (g.n - g.batch + g.n_batches - 1) / g.n_batches;
    const int gw = (blockIdx.x * blockDim.x + tid) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    for (int idx = gw; idx < nbc; idx += nw) {
        const int v = g.batch + idx * g.n_batches;
        const int x = nb[v];
        if (x < 0) continue;
        const int r = g.lab[v];
        const int op = g.out_ptr[v], kout = g.out_ptr[v + 1] - op;
        const int ip = g.in_ptr[v], kin = g.in_ptr[v + 1] - ip;
        for (int j = lane; j < kout; j += 64) {  // out-edges: counted here
            const int w = g.out_idx[op + j];
            const int b = g.lab[w];
            const bool wmoved = (w % g.n_batches) == g.batch && nb[w] >= 0;
            const int b2 = wmoved ? nb[w] : b;
            atomicAdd(&dl[r * C + b], -1);
            atomicAdd(&dl[x * C + b2], 1);
        }
        for (int j = lane; j < kin; j += 64) {  // in-edges from sources that stayed
            const int u = g.in_idx[ip + j];
            if ((u % g.n_batches) == g.batch && nb[u] >= 0) continue;
            const int a = g.lab[u];
            atomicAdd(&dl[a * C + r], -1);
            atomicAdd(&dl[a * C + x], 1);
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
    hipLaunchKernelGGL(k_dense_hist, dim3(grid_for(g.n, 256, 1024)), dim3(256), 0, s, g, bm.M);
    hipLaunchKernelGGL(k_dense_final, dim3(1), dim3(1024), 0, s, g, bm, (const long long *)nullptr,
                       (const double *)nullptr, 0, (sbp_sweep_stats_dev *)nullptr);
    SBP_LAUNCH_CHECK();
    return 0;
}

int dense_sweep_batch(const GDev &g, DenseBM &bm, DenseScratch &ws, const SweepTraceDev &tr,
                      sbp_sweep_stats_dev *stats, hipStream_t s) {
    const int nbc = (g.n - g.batch + g.n_batches - 1) / g.n_batches;
    int grid = (nbc + EVAL_WAVES - 1) / EVAL_WAVES;
    if (grid > ws.nwg) grid = ws.nwg;
    if (grid < 1) grid = 1;
    {
        ProfileScope prof("sweep_eval", s);
        hipLaunchKernelGGL(k_dense_eval, dim3(grid), dim3(EVAL_WAVES * 64), 0, s, g, bm, ws.nb, tr, ws.stats_part,
                           ws.sum_part);
    }
    hipLaunchKernelGGL(k_dense_delta, dim3(grid), dim3(256), 0, s, g, (const int *)ws.nb, ws.delta);
    hipLaunchKernelGGL(k_dense_apply, dim3(grid_for(g.C * g.C + nbc, 256, 2048)), dim3(256), 0, s, g, bm, ws.delta,
                       ws.nb);
    hipLaunchKernelGGL(k_dense_final, dim3(1), dim3(1024), 0, s, g, bm, ws.stats_part, ws.sum_part, grid, stats);
    SBP_LAUNCH_CHECK();
    return 0;
}

int dense_merge_scores(const GDev &g, const DenseBM &bm, int *partner, double *dS, double *dSl, hipStream_t s) {
    hipLaunchKernelGGL(k_dense_merge, dim3((g.C * 64 + 255) / 256), dim3(256), 0, s, g, bm, partner, dS, dSl);
    SBP_LAUNCH_CHECK();
    return 0;
}

}  // namespace sbp
