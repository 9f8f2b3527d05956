// sbp_prims.hip -- device-wide exclusive scan and stable LSD radix sort for gfx950.
//
// Scan: three kernels (tile reduce, scan of tile sums in one workgroup, tile
// scan plus offset).  Radix sort: 8-bit digits; per pass a tile histogram,
// a scan of the digit-major histogram, and a stable scatter whose in-tile
// ranks come from wave64 ballots (lanes with an equal digit are found with
// eight ballots, ranks are popcounts below the lane).
#include "sbp_internal.h"

namespace sbp {

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

template <class T>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_reduce(const T *__restrict__ in, long long n,
                                                           long long *__restrict__ tile_sum) {
    __shared__ long long wsum[SCAN_BLOCK / SBP_WAVE];
    const long long base = (long long)blockIdx.x * SCAN_TILE;
    long long acc = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const long long idx = base + (long long)i * SCAN_BLOCK + threadIdx.x;
        if (idx < n) acc += (long long)in[idx];
    }
    acc = wave_sum_i64(acc);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int w = 0; w < SCAN_BLOCK / SBP_WAVE; ++w) t += wsum[w];
        tile_sum[blockIdx.x] = t;
    }
}

// Exclusive scan of the tile sums in one workgroup (sequential chunks of 1024).
__global__ void __launch_bounds__(1024) k_scan_tiles(long long *__restrict__ tile_sum, long long ntiles,
                                                     long long *__restrict__ total) {
    __shared__ long long wpre[1024 / SBP_WAVE];
    __shared__ long long carry_s;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (long long base = 0; base < ntiles; base += 1024) {
        const long long idx = base + threadIdx.x;
        const long long v = idx < ntiles ? tile_sum[idx] : 0;
        // inclusive scan within the wave
        long long x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const long long y = __shfl_up(x, o, SBP_WAVE);
            if (lane >= o) x += y;
        }
        if (lane == 63) wpre[wave] = x;
        __syncthreads();
        if (threadIdx.x == 0) {
            long long run = 0;
            for (int w = 0; w < 1024 / SBP_WAVE; ++w) {
                const long long t = wpre[w];
                wpre[w] = run;
                run += t;
            }
        }
        __syncthreads();
        const long long carry = carry_s;
        if (idx < ntiles) tile_sum[idx] = carry + wpre[wave] + x - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry_s = carry + wpre[wave] + x;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry_s;
}

template <class T>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_down(const T *__restrict__ in, long long n,
                                                         const long long *__restrict__ tile_off,
                                                         long long *__restrict__ out) {
    __shared__ long long wpre[SCAN_BLOCK / SBP_WAVE];
    const long long base = (long long)blockIdx.x * SCAN_TILE;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // blocked arrangement: thread t owns items [t*ITEMS, (t+1)*ITEMS) of the tile
    long long v[SCAN_ITEMS];
    long long run = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const long long idx = base + (long long)threadIdx.x * SCAN_ITEMS + i;
        v[i] = idx < n ? (long long)in[idx] : 0;
        run += v[i];
    }
    long long x = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long y = __shfl_up(x, o, SBP_WAVE);
        if (lane >= o) x += y;
    }
    if (lane == 63) wpre[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long r = 0;
        for (int w = 0; w < SCAN_BLOCK / SBP_WAVE; ++w) {
            const long long t = wpre[w];
            wpre[w] = r;
            r += t;
        }
    }
    __syncthreads();
    long long pre = tile_off[blockIdx.x] + wpre[wave] + x - run;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const long long idx = base + (long long)threadIdx.x * SCAN_ITEMS + i;
        if (idx < n) out[idx] = pre;
        pre += v[i];
    }
}

template <class T>
int scan_exclusive_t(const T *in, long long *out, long long n, long long *total, void *temp, hipStream_t s) {
    if (n <= 0) {
        if (total) {
            hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, (long long *)temp, 0LL, total);
            SBP_LAUNCH_CHECK();
        }
        return 0;
    }
    const long long ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    long long *tiles = (long long *)temp;
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)ntiles), dim3(SCAN_BLOCK), 0, s, in, n, tiles);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, tiles, ntiles, total);
    hipLaunchKernelGGL(k_scan_down<T>, dim3((unsigned)ntiles), dim3(SCAN_BLOCK), 0, s, in, n, tiles, out);
    SBP_LAUNCH_CHECK();
    return 0;
}

// ---------------------------------------------------------------- radix sort
constexpr int RADIX_BLOCK = 256;
constexpr int RADIX_ITEMS = 8;
constexpr int RADIX_TILE = RADIX_BLOCK * RADIX_ITEMS;
constexpr int RADIX_DIGITS = 256;

__global__ void __launch_bounds__(RADIX_BLOCK) k_radix_hist(const uint64_t *__restrict__ keys, long long n, int shift,
                                                           long long ntiles, int *__restrict__ hist) {
    __shared__ int h[RADIX_DIGITS];
    h[threadIdx.x] = 0;
    __syncthreads();
    const long long base = (long long)blockIdx.x * RADIX_TILE;
#pragma unroll
    for (int i = 0; i < RADIX_ITEMS; ++i) {
        const long long idx = base + (long long)i * RADIX_BLOCK + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 0xFF], 1);
    }
    __syncthreads();
    hist[(long long)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// One tile of the stable scatter: ranks as in the wave-ballot scheme (keys of
// equal digit keep their order), but each key first goes to its digit's run
// in an LDS copy of the tile; the tile is then written out in LDS order, so
// a run of equal digits lands in consecutive global slots.
template <bool VALS>
__global__ void __launch_bounds__(RADIX_BLOCK) k_radix_scatter(const uint64_t *__restrict__ kin,
                                                              const uint64_t *__restrict__ vin,
                                                              uint64_t *__restrict__ kout,
                                                              uint64_t *__restrict__ vout, long long n, int shift,
                                                              long long ntiles, const long long *__restrict__ off,
                                                              const int *__restrict__ hist) {
    constexpr int NW = RADIX_BLOCK / SBP_WAVE;
    __shared__ long long goff[RADIX_DIGITS];
    __shared__ int loff[RADIX_DIGITS];
    __shared__ int run[RADIX_DIGITS];
    __shared__ int wcnt[NW][RADIX_DIGITS];
    __shared__ int wpre[NW][RADIX_DIGITS];
    __shared__ uint64_t sk[RADIX_TILE];
    __shared__ uint64_t sv[VALS ? RADIX_TILE : 1];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    goff[t] = off[(long long)t * ntiles + blockIdx.x];
    run[t] = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) wcnt[w][t] = 0;
    // tile-local start of every digit: exclusive scan of the tile's counts
    {
        const int c = hist[(long long)t * ntiles + blockIdx.x];
        int x = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, SBP_WAVE);
            if (lane >= o) x += y;
        }
        if (lane == 63) wpre[0][wave] = x;
        __syncthreads();
        int before = 0;
        for (int w = 0; w < wave; ++w) before += wpre[0][w];
        loff[t] = before + x - c;
    }
    __syncthreads();
    const long long base = (long long)blockIdx.x * RADIX_TILE;
    const int tn = (int)min((long long)RADIX_TILE, n - base);
    const uint64_t below = lanemask_lt();
    for (int i = 0; i < RADIX_ITEMS; ++i) {
        const int li = i * RADIX_BLOCK + t;
        const bool valid = li < tn;
        uint64_t key = 0, val = 0;
        if (valid) {
            key = kin[base + li];
            if (VALS) val = vin[base + li];
        }
        const unsigned d = (unsigned)((key >> shift) & 0xFF);
        uint64_t eq = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            eq &= bit ? m : ~m;
        }
        const int rank = __popcll(eq & below);
        if (valid && rank == 0) wcnt[wave][d] = __popcll(eq);
        __syncthreads();
        {
            int r = run[t];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const int c = wcnt[w][t];
                wpre[w][t] = r;
                r += c;
                wcnt[w][t] = 0;
            }
            run[t] = r;
        }
        __syncthreads();
        if (valid) {
            const int pos = loff[d] + wpre[wave][d] + rank;
            sk[pos] = key;
            if (VALS) sv[pos] = val;
        }
        __syncthreads();
    }
    for (int li = t; li < tn; li += RADIX_BLOCK) {
        const uint64_t key = sk[li];
        const unsigned d = (unsigned)((key >> shift) & 0xFF);
        const long long pos = goff[d] + (li - loff[d]);
        kout[pos] = key;
        if (VALS) vout[pos] = sv[li];
    }
}

__global__ void k_fill_i32(int *p, int value, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = value;
}
__global__ void k_fill_i64(long long *p, long long value, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = value;
}
__global__ void k_iota_i32(int *p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = (int)i;
}

}  // namespace

size_t scan_temp_bytes(long long n) { return (size_t)((n + SCAN_TILE - 1) / SCAN_TILE + 2) * sizeof(long long); }

int scan_exclusive_i32(const int *in, long long *out, long long n, long long *total, void *temp, hipStream_t s) {
    return scan_exclusive_t<int>(in, out, n, total, temp, s);
}
int scan_exclusive_i64(const long long *in, long long *out, long long n, long long *total, void *temp,
                       hipStream_t s) {
    return scan_exclusive_t<long long>(in, out, n, total, temp, s);
}

size_t radix_temp_bytes(long long n) {
    const long long ntiles = (n + RADIX_TILE - 1) / RADIX_TILE;
    const long long h = ntiles * RADIX_DIGITS;
    // histogram (int) + offsets (int64) + scan temp
    return (size_t)(h * sizeof(int) + 256) + (size_t)(h * sizeof(long long) + 256) + scan_temp_bytes(h) + 256;
}

int radix_sort(uint64_t *keys, uint64_t *keys_alt, uint64_t *vals, uint64_t *vals_alt, long long n, int bits,
               void *temp, hipStream_t s) {
    return radix_sort_bits(keys, keys_alt, vals, vals_alt, n, 0, bits, temp, s);
}

int radix_sort_bits(uint64_t *keys, uint64_t *keys_alt, uint64_t *vals, uint64_t *vals_alt, long long n, int lo,
                    int bits, void *temp, hipStream_t s) {
    if (n <= 1 || bits <= lo) return 0;
    const long long ntiles = (n + RADIX_TILE - 1) / RADIX_TILE;
    const long long h = ntiles * RADIX_DIGITS;
    char *t = (char *)temp;
    int *hist = (int *)t;
    t += ((h * sizeof(int) + 255) & ~255ll) + 256;
    long long *off = (long long *)t;
    t += ((h * sizeof(long long) + 255) & ~255ll) + 256;
    void *stemp = t;
    uint64_t *ka = keys, *kb = keys_alt, *va = vals, *vb = vals_alt;
    int passes = 0;
    for (int shift = lo; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)ntiles), dim3(RADIX_BLOCK), 0, s, ka, n, shift, ntiles, hist);
        SBP_LAUNCH_CHECK();
        int rc = scan_exclusive_i32(hist, off, h, nullptr, stemp, s);
        if (rc) return rc;
        if (vals)
            hipLaunchKernelGGL(k_radix_scatter<true>, dim3((unsigned)ntiles), dim3(RADIX_BLOCK), 0, s, ka, va, kb, vb,
                               n, shift, ntiles, off, hist);
        else
            hipLaunchKernelGGL(k_radix_scatter<false>, dim3((unsigned)ntiles), dim3(RADIX_BLOCK), 0, s, ka, va, kb,
                               vb, n, shift, ntiles, off, hist);
        SBP_LAUNCH_CHECK();
        uint64_t *x = ka; ka = kb; kb = x;
        x = va; va = vb; vb = x;
        ++passes;
    }
    if (passes & 1) {
        SBP_HIP_CHECK(hipMemcpyAsync(keys, ka, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        if (vals) SBP_HIP_CHECK(hipMemcpyAsync(vals, va, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    }
    return 0;
}

int fill_i32(int *p, int value, long long n, hipStream_t s) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, value, n);
    SBP_LAUNCH_CHECK();
    return 0;
}
int fill_i64(long long *p, long long value, long long n, hipStream_t s) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, value, n);
    SBP_LAUNCH_CHECK();
    return 0;
}
int iota_i32(int *p, long long n, hipStream_t s) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_iota_i32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n);
    SBP_LAUNCH_CHECK();
    return 0;
}

}  // namespace sbp
