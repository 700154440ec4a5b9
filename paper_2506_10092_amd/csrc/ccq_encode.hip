// Encoding on the device (Table 1: plain_to_rle, plain_to_rle+index,
// plain_to_plain+index) and the encoding choice of the evaluation setup
// (Section 9: Plain under 1M rows, RLE above a compression ratio of 20,
// RLE+Index when single-row runs spoil RLE, Plain+Index when cutting the top
// and bottom 5% of values narrows the type, else centered Plain).
//
// Every encoder is a stream compaction: a per-row flag says whether the row
// starts a run, ends one, or is an outlier; output slots are the flag's rank
// among all rows.  A wavefront takes 1024-row chunks: each lane loads 16
// rows, one coalesced wave load each (row r0 + 64 k + lane), finds its
// rows' neighbours with lane shuffles, and ballots rank the chunk's flags,
// with no LDS and no barrier.  Launch sequence per encoder: count (flag
// totals per chunk), a three-kernel scan (exclusive offsets per chunk),
// write (the same pass again, writing at the offsets).  The order
// statistics of the choice come from a radix select: eight passes of 8-bit
// digit histograms over the order-preserving 64-bit keys, each pass keeping
// the digit that holds the wanted rank.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "ccq_internal.h"

namespace ccq {
namespace {

constexpr int kEncThreads = 256;
constexpr int kEncRowsPerThread = 16;
constexpr int64_t kChooseMinRows = 1000000;   // columns under this many rows stay Plain
constexpr double kChooseRatio = 20.0;          // compression ratio that selects RLE / RLE+Index

__device__ __forceinline__ int64_t load_value(const void* v, int32_t vtype, int64_t i) {
    return vtype == CCQ_I32 ? (int64_t)((const int32_t*)v)[i] : ((const int64_t*)v)[i];
}

__device__ __forceinline__ void store_value(void* v, int32_t vtype, int64_t i, int64_t x) {
    if (vtype == CCQ_I32) ((int32_t*)v)[i] = (int32_t)x;
    else ((int64_t*)v)[i] = x;
}

// inclusive prefix sum over the workgroup's threads (all threads call)
__device__ __forceinline__ int64_t block_inclusive_sum(int64_t x, int64_t* s_wave, int64_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int w = 0; w < kEncThreads / 64; ++w) {
        const int64_t t = s_wave[w];
        if (w < wave) before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return x + before;
}

enum EncMode : int32_t { kModeRle = 0, kModeRleIndex = 1, kModePlainIndex = 2 };

// Rows go in wave chunks of kWaveChunk rows: lane l holds rows
// r0 + 64 k + l for k < kEncRowsPerThread, so each of a lane's loads is one
// coalesced wave load, a row's neighbours come from the next or previous
// lane (or, across lanes 0 and 63, the neighbouring k or chunk), and row
// order within the chunk is (k, lane), in which ballots rank the flags.
constexpr int kWaveChunk = 64 * kEncRowsPerThread;      // 1024 rows

struct EncArgs {
    const void* values;
    int32_t vtype;
    int32_t mode;
    int64_t n;
    // plain+index: codes in [0, 2^w) above base stay plain
    int64_t base;
    int32_t w;
    int32_t out_vtype;
    // outputs (write pass)
    void* run_values;       // RLE, RLE+Index: run values
    int64_t* run_starts;    // RLE+Index: run starts
    int64_t* run_ends;      // RLE, RLE+Index: exclusive run ends
    int64_t* idx_pos;       // RLE+Index, Plain+Index: point positions
    void* idx_vals;         // point values
    int32_t* cnt;           // [2][n_wc]: flags 0 and 1 per wave chunk
    const int64_t* off;     // [2][n_wc + 1]: exclusive offsets per wave chunk
    int64_t n_wc;
};

// One wave chunk: the lane's rows, their two flags (flag 0 ranks runs --
// RLE: every run start; RLE+Index: starts of runs of two or more rows;
// Plain+Index: outliers -- flag 1 the points of RLE+Index, rows that form a
// run of their own) and, with WRITE, the outputs at the ranks from o0, o1.
// Returns the chunk's flag counts (wave-uniform).
// T: the column's value type (int32_t or int64_t), so int32 columns shuffle
// and compare 32-bit values.
template <typename T, bool WRITE>
__device__ __forceinline__ void wave_chunk(const EncArgs& A, int64_t wc, int64_t o0, int64_t o1, int32_t* c0,
                                           int32_t* c1) {
    const int lane = threadIdx.x & 63;
    const int64_t r0 = wc * kWaveChunk;
    const T* v = (const T*)A.values;
    T x[kEncRowsPerThread];
#pragma unroll
    for (int k = 0; k < kEncRowsPerThread; ++k) {
        const int64_t i = r0 + 64 * k + lane;
        x[k] = i < A.n ? v[i] : T(0);
    }
    const T before = r0 > 0 ? v[r0 - 1] : T(0);
    const T after = r0 + kWaveChunk < A.n ? v[r0 + kWaveChunk] : T(0);
    const uint64_t below = (1ull << lane) - 1ull;
    int32_t n0 = 0, n1 = 0;
#pragma unroll
    for (int k = 0; k < kEncRowsPerThread; ++k) {
        const int64_t i = r0 + 64 * k + lane;
        const T xi = x[k];
        T prev = __shfl_up(xi, 1, 64);
        T next = __shfl_down(xi, 1, 64);
        const T last_prev = k > 0 ? __shfl(x[k - 1], 63, 64) : before;
        const T first_next = k + 1 < kEncRowsPerThread ? __shfl(x[k + 1 < kEncRowsPerThread ? k + 1 : k], 0, 64)
                                                        : after;
        if (lane == 0) prev = last_prev;
        if (lane == 63) next = first_next;
        const bool valid = i < A.n;
        const bool start = valid && (i == 0 || xi != prev);
        const bool end = valid && (i == A.n - 1 || xi != next);
        bool f0, f1;
        if (A.mode == kModeRle) {
            f0 = start;
            f1 = false;
        } else if (A.mode == kModeRleIndex) {
            f0 = start && !end;
            f1 = start && end;
        } else {
            // outside [base, base + 2^w); once x >= base the wrapped difference is exact
            const uint64_t code = (uint64_t)(int64_t)xi - (uint64_t)A.base;
            f0 = valid && ((int64_t)xi < A.base || (code >> A.w) != 0);
            f1 = false;
        }
        const uint64_t m0 = __ballot(f0), m1 = __ballot(f1);
        if constexpr (WRITE) {
            const int64_t ra = o0 + n0 + __builtin_popcountll(m0 & below);   // rank of this row's flag 0
            const int64_t rb = o1 + n1 + __builtin_popcountll(m1 & below);
            if (A.mode == kModeRle) {
                if (f0) store_value(A.run_values, A.out_vtype, ra, xi);
                // the run holding row i is the last one started at or before it
                if (end) A.run_ends[ra + (f0 ? 1 : 0) - 1] = i + 1;
            } else if (A.mode == kModeRleIndex) {
                if (f0) {
                    store_value(A.run_values, A.out_vtype, ra, xi);
                    A.run_starts[ra] = i;
                }
                if (end && !start) A.run_ends[ra - 1] = i + 1;   // the end of a run of two or more rows
                if (f1) {
                    A.idx_pos[rb] = i;
                    store_value(A.idx_vals, A.out_vtype, rb, xi);
                }
            } else if (f0) {
                A.idx_pos[ra] = i;
                store_value(A.idx_vals, A.out_vtype, ra, xi);
            }
        }
        n0 += __builtin_popcountll(m0);
        n1 += __builtin_popcountll(m1);
    }
    *c0 = n0;
    *c1 = n1;
}

// flag counts per wave chunk (a wave per chunk, grid-stride)
template <typename T>
__global__ __launch_bounds__(kEncThreads) void k_enc_count(EncArgs A) {
    const int64_t waves = (int64_t)gridDim.x * (kEncThreads / 64);
    for (int64_t wc = (int64_t)blockIdx.x * (kEncThreads / 64) + (threadIdx.x >> 6); wc < A.n_wc; wc += waves) {
        int32_t c0, c1;
        wave_chunk<T, false>(A, wc, 0, 0, &c0, &c1);
        if ((threadIdx.x & 63) == 0) {
            A.cnt[wc] = c0;
            A.cnt[A.n_wc + wc] = c1;
        }
    }
}

// ---- exclusive scan of the per-chunk counts (int32) into int64 offsets

constexpr int64_t kEncScanPer = 4096;

// per part of kEncScanPer counts: its total (flag f = blockIdx.y)
__global__ __launch_bounds__(kEncThreads) void k_enc_scan_part(const int32_t* cnt, int64_t n, int64_t* part,
                                                               int64_t n_parts) {
    __shared__ int64_t s_wave[kEncThreads / 64];
    const int32_t* c = cnt + blockIdx.y * n;
    const int64_t p0 = (int64_t)blockIdx.x * kEncScanPer;
    int64_t x = 0;
    for (int64_t i = p0 + threadIdx.x; i < min(n, p0 + kEncScanPer); i += kEncThreads) x += c[i];
    int64_t t;
    block_inclusive_sum(x, s_wave, &t);
    if (threadIdx.x == 0) part[blockIdx.y * (n_parts + 1) + blockIdx.x] = t;
}

// exclusive scan of the part totals in place, the grand total at part[n_parts] (one workgroup per flag)
__global__ __launch_bounds__(kEncThreads) void k_enc_scan_parts(int64_t* part, int64_t n_parts) {
    __shared__ int64_t s_wave[kEncThreads / 64];
    int64_t* p = part + blockIdx.y * (n_parts + 1);
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < n_parts; b0 += kEncThreads) {
        const int64_t b = b0 + threadIdx.x;
        const int64_t x = b < n_parts ? p[b] : 0;
        int64_t all;
        const int64_t inc = block_inclusive_sum(x, s_wave, &all);
        if (b < n_parts) p[b] = carry + inc - x;
        carry += all;
    }
    if (threadIdx.x == 0) p[n_parts] = carry;
}

// off[f][i] = the part's offset plus the in-part exclusive scan; off[f][n] = the total
__global__ __launch_bounds__(kEncThreads) void k_enc_scan_final(const int32_t* cnt, int64_t n, const int64_t* part,
                                                                int64_t n_parts, int64_t* off) {
    __shared__ int64_t s_wave[kEncThreads / 64];
    const int32_t* c = cnt + blockIdx.y * n;
    const int64_t* p = part + blockIdx.y * (n_parts + 1);
    int64_t* o = off + blockIdx.y * (n + 1);
    const int64_t p0 = (int64_t)blockIdx.x * kEncScanPer;
    int64_t carry = p[blockIdx.x];
    for (int64_t b0 = p0; b0 < min(n, p0 + kEncScanPer); b0 += kEncThreads) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t x = i < n ? c[i] : 0;
        int64_t all;
        const int64_t inc = block_inclusive_sum(x, s_wave, &all);
        if (i < n) o[i] = carry + inc - x;
        carry += all;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) o[n] = p[n_parts];
}

// the outputs, each wave chunk at its offsets
template <typename T>
__global__ __launch_bounds__(kEncThreads) void k_enc_write(EncArgs A) {
    const int64_t waves = (int64_t)gridDim.x * (kEncThreads / 64);
    for (int64_t wc = (int64_t)blockIdx.x * (kEncThreads / 64) + (threadIdx.x >> 6); wc < A.n_wc; wc += waves) {
        int32_t c0, c1;
        wave_chunk<T, true>(A, wc, A.off[wc], A.off[A.n_wc + 1 + wc], &c0, &c1);
    }
}

// Plain+Index codes: thread t packs rows [32t, 32t + 32) into its w words
// (value - base, 0 for outliers), LSB-first, row r at bits [r w, r w + w).
// Fewer than 32 bits are pending before each code is added and w <= 32, so a
// 64-bit accumulator never drops a bit.
__global__ __launch_bounds__(kEncThreads) void k_enc_pack(const void* v, int32_t vtype, int64_t n, int64_t base,
                                                           int32_t w, uint32_t* packed, int64_t n_words) {
    const int64_t lw = (int64_t)blockIdx.x * kEncThreads + threadIdx.x;
    const int64_t r0 = lw * 32;
    if (r0 >= n) return;
    const uint64_t lim = w == 32 ? 0xFFFFFFFFull : ((1ull << w) - 1ull);
    uint64_t acc = 0;
    int nacc = 0;
    int64_t word = lw * w;
    for (int k = 0; k < 32; ++k) {
        const int64_t i = r0 + k;
        uint64_t code = 0;
        if (i < n) {
            const int64_t x = load_value(v, vtype, i);
            code = (uint64_t)x - (uint64_t)base;
            if (x < base || code > lim) code = 0;   // an outlier: its value is in the Index part
        }
        acc |= code << nacc;
        nacc += w;
        if (nacc >= 32) {
            if (word < n_words) packed[word] = (uint32_t)acc;
            ++word;
            acc >>= 32;
            nacc -= 32;
        }
    }
}

// Column statistics: maximal runs, runs of one row, min and max (i < n).
struct EncStats {
    unsigned long long runs, singles;
    long long vmin, vmax;
};

template <typename T>
__global__ __launch_bounds__(kEncThreads) void k_enc_stats(const void* v, int32_t vtype, int64_t n, EncStats* out) {
    // runs and single-row runs: flags 0 and 1 of RLE+Index, per wave chunk
    EncArgs A = {};
    A.values = v;
    A.vtype = vtype;
    A.mode = kModeRleIndex;
    A.n = n;
    A.n_wc = (n + kWaveChunk - 1) / kWaveChunk;
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (kEncThreads / 64);
    int64_t runs = 0, singles = 0, lo = INT64_MAX, hi = INT64_MIN;
    for (int64_t wc = (int64_t)blockIdx.x * (kEncThreads / 64) + (threadIdx.x >> 6); wc < A.n_wc; wc += waves) {
        int32_t c0, c1;
        wave_chunk<T, false>(A, wc, 0, 0, &c0, &c1);
        runs += c0 + c1;
        singles += c1;
        for (int k = 0; k < kEncRowsPerThread; ++k) {
            const int64_t i = wc * kWaveChunk + 64 * k + lane;
            if (i < n) {
                const int64_t x = load_value(v, vtype, i);
                lo = min(lo, x);
                hi = max(hi, x);
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, (int64_t)__shfl_xor(lo, o, 64));
        hi = max(hi, (int64_t)__shfl_xor(hi, o, 64));
    }
    if (lane == 0) {
        atomicMin(&out->vmin, (long long)lo);
        atomicMax(&out->vmax, (long long)hi);
        atomicAdd(&out->runs, (unsigned long long)runs);      // wave-uniform counts, one add per wave
        atomicAdd(&out->singles, (unsigned long long)singles);
    }
}

__global__ void k_enc_stats_init(EncStats* out) {
    out->runs = 0;
    out->singles = 0;
    out->vmin = INT64_MAX;
    out->vmax = INT64_MIN;
}

// Radix select: 8-bit digit histograms at bit `shift` of the order-preserving
// keys (value ^ 2^63) of the rows whose key agrees with prefix[t] above the
// digit, for two wanted ranks t = 0, 1 at once.  hist: [2][256], cleared by
// the host before each pass.
__global__ __launch_bounds__(kEncThreads) void k_enc_hist(const void* v, int32_t vtype, int64_t n, int32_t shift,
                                                           uint64_t prefix0, uint64_t prefix1,
                                                           unsigned long long* hist) {
    __shared__ unsigned int h[2][256];
    for (int k = threadIdx.x; k < 512; k += kEncThreads) h[k >> 8][k & 255] = 0;
    __syncthreads();
    const int hs = shift + 8;
    const int64_t stride = (int64_t)gridDim.x * kEncThreads;
    for (int64_t i = (int64_t)blockIdx.x * kEncThreads + threadIdx.x; i < n; i += stride) {
        const uint64_t key = (uint64_t)load_value(v, vtype, i) ^ (1ull << 63);
        const uint64_t above = hs >= 64 ? 0 : key >> hs;
        const unsigned d = (unsigned)(key >> shift) & 255u;
        if (above == prefix0) atomicAdd(&h[0][d], 1u);
        if (above == prefix1) atomicAdd(&h[1][d], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 512; k += kEncThreads)
        if (h[k >> 8][k & 255]) atomicAdd(&hist[k], (unsigned long long)h[k >> 8][k & 255]);
}

int bits_for(uint64_t x) { return x == 0 ? 1 : 64 - __builtin_clzll(x); }

struct EncWs {
    int64_t n_wc;               // wave chunks
    int64_t n_parts;            // scan parts
    unsigned grid;              // workgroups of the chunk kernels
    int32_t* cnt;               // [2][n_wc]
    int64_t* off;               // [2][n_wc + 1]
    int64_t* part;              // [2][n_parts + 1]
    EncStats* stats;
    unsigned long long* hist;   // [2][256]
};

size_t a256e(size_t x) { return (x + 255) & ~size_t(255); }

EncWs enc_ws(void* ws, int64_t n) {
    EncWs w;
    w.n_wc = std::max<int64_t>(1, (n + kWaveChunk - 1) / kWaveChunk);
    w.n_parts = (w.n_wc + kEncScanPer - 1) / kEncScanPer;
    w.grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((w.n_wc + 3) / 4, 8192));
    unsigned char* p = (unsigned char*)ws;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        unsigned char* q = p ? p + o : nullptr;
        o += a256e(bytes);
        return q;
    };
    w.stats = (EncStats*)take(sizeof(EncStats));
    w.hist = (unsigned long long*)take(4096);
    w.cnt = (int32_t*)take(4 * 2 * (size_t)w.n_wc);
    w.off = (int64_t*)take(8 * 2 * (size_t)(w.n_wc + 1));
    w.part = (int64_t*)take(8 * 2 * (size_t)(w.n_parts + 1));
    return w;
}

size_t enc_ws_bytes(int64_t n) {
    // the layout's size: enc_ws over a null base, the last piece's end
    const EncWs w = enc_ws(nullptr, n);
    return a256e(sizeof(EncStats)) + 4096 + a256e(4 * 2 * (size_t)w.n_wc) + a256e(8 * 2 * (size_t)(w.n_wc + 1)) +
           a256e(8 * 2 * (size_t)(w.n_parts + 1));
}

ccq_status enc_check(ccq_context* ctx, const void* values, int32_t vtype, int64_t n, void* ws, size_t ws_bytes) {
    if (!ctx || ctx->device < 0) return fail(CCQ_E_INVALID, "a device context is required");
    if (vtype != CCQ_I32 && vtype != CCQ_I64) return fail(CCQ_E_INVALID, "value_type must be CCQ_I32 or CCQ_I64");
    if (n < 0) return fail(CCQ_E_INVALID, "n_rows must be >= 0");
    if (n > 0 && !values) return fail(CCQ_E_INVALID, "values missing");
    if (!ws || ((uintptr_t)ws & 255)) return fail(CCQ_E_INVALID, "workspace must be 256-byte aligned");
    if (ws_bytes < enc_ws_bytes(n))
        return fail(CCQ_E_CAPACITY, "workspace of %zu bytes, %zu needed", ws_bytes, enc_ws_bytes(n));
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return CCQ_OK;
}

void launch_write(const EncArgs& A, const EncWs& w, hipStream_t s) {
    if (A.vtype == CCQ_I32) hipLaunchKernelGGL(k_enc_write<int32_t>, dim3(w.grid), dim3(kEncThreads), 0, s, A);
    else hipLaunchKernelGGL(k_enc_write<int64_t>, dim3(w.grid), dim3(kEncThreads), 0, s, A);
}

// count + scan for one mode; returns the two flag totals (synchronises)
ccq_status enc_count(EncArgs& A, const EncWs& w, hipStream_t s, int64_t* t0, int64_t* t1) {
    A.cnt = w.cnt;
    A.off = w.off;
    A.n_wc = w.n_wc;
    if (A.vtype == CCQ_I32) hipLaunchKernelGGL(k_enc_count<int32_t>, dim3(w.grid), dim3(kEncThreads), 0, s, A);
    else hipLaunchKernelGGL(k_enc_count<int64_t>, dim3(w.grid), dim3(kEncThreads), 0, s, A);
    hipLaunchKernelGGL(k_enc_scan_part, dim3((unsigned)w.n_parts, 2), dim3(kEncThreads), 0, s, w.cnt, w.n_wc, w.part,
                       w.n_parts);
    hipLaunchKernelGGL(k_enc_scan_parts, dim3(1, 2), dim3(kEncThreads), 0, s, w.part, w.n_parts);
    hipLaunchKernelGGL(k_enc_scan_final, dim3((unsigned)w.n_parts, 2), dim3(kEncThreads), 0, s, w.cnt, w.n_wc,
                       w.part, w.n_parts, w.off);
    int64_t h[2];
    hipError_t e = hipMemcpyAsync(&h[0], w.off + w.n_wc, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&h[1], w.off + 2 * w.n_wc + 1, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "encode count");
    *t0 = h[0];
    *t1 = h[1];
    return CCQ_OK;
}

}  // namespace
}  // namespace ccq

using namespace ccq;

extern "C" {

size_t ccq_encode_workspace_bytes(int64_t n_rows) { return enc_ws_bytes(std::max<int64_t>(n_rows, 0)); }

ccq_status ccq_encode_choose(ccq_context* ctx, const void* values, int32_t value_type, int64_t n_rows, void* ws,
                             size_t ws_bytes, void* stream, ccq_encoding_choice* out) {
    if (!out) return fail(CCQ_E_INVALID, "out is NULL");
    if (ccq_status st = enc_check(ctx, values, value_type, n_rows, ws, ws_bytes)) return st;
    hipStream_t s = (hipStream_t)stream;
    memset(out, 0, sizeof *out);
    out->n_rows = n_rows;
    if (n_rows == 0) {
        out->choice = CCQ_CHOOSE_PLAIN;
        out->bit_width = 1;
        return ok();
    }
    const EncWs w = enc_ws(ws, n_rows);
    hipLaunchKernelGGL(k_enc_stats_init, dim3(1), dim3(1), 0, s, w.stats);
    hipLaunchKernelGGL(value_type == CCQ_I32 ? k_enc_stats<int32_t> : k_enc_stats<int64_t>, dim3(w.grid),
                       dim3(kEncThreads), 0, s, values, value_type, n_rows,
                       w.stats);
    EncStats st;
    hipError_t e = hipMemcpyAsync(&st, w.stats, sizeof st, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "encode statistics");
    out->runs = (int64_t)st.runs;
    out->single_runs = (int64_t)st.singles;
    out->min_value = st.vmin;
    out->max_value = st.vmax;

    // the values at sorted ranks floor(n / 20) and n - 1 - floor(n / 20)
    int64_t rank[2] = {n_rows / 20, n_rows - 1 - n_rows / 20};
    uint64_t prefix[2] = {0, 0};
    const unsigned hgrid = (unsigned)std::min<int64_t>((n_rows + kEncThreads - 1) / kEncThreads, 4096);
    for (int shift = 56; shift >= 0; shift -= 8) {
        e = hipMemsetAsync(w.hist, 0, 512 * sizeof(unsigned long long), s);
        if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
        hipLaunchKernelGGL(k_enc_hist, dim3(hgrid), dim3(kEncThreads), 0, s, values, value_type, n_rows, shift,
                           prefix[0], prefix[1], w.hist);
        unsigned long long h[512];
        e = hipMemcpyAsync(h, w.hist, sizeof h, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "encode select");
        for (int t = 0; t < 2; ++t) {
            int d = 0;
            while (d < 255 && rank[t] >= (int64_t)h[t * 256 + d]) rank[t] -= (int64_t)h[t * 256 + d++];
            prefix[t] = (prefix[t] << 8) | (uint64_t)d;
        }
    }
    out->lo_cut = (int64_t)(prefix[0] ^ (1ull << 63));
    out->hi_cut = (int64_t)(prefix[1] ^ (1ull << 63));

    // The choice.  A run costs three elements (value, start, end) as in the
    // paper's representation; RLE+Index is taken when single-row runs exist
    // and the longer runs alone still compress by more than 20.
    const double vb = value_type == CCQ_I32 ? 4.0 : 8.0;
    const double plain_bytes = (double)n_rows * vb;
    const int64_t longs = out->runs - out->single_runs;
    const int w_full = bits_for((uint64_t)out->max_value - (uint64_t)out->min_value);
    const int w_cut = bits_for((uint64_t)out->hi_cut - (uint64_t)out->lo_cut);
    if (n_rows >= kChooseMinRows && plain_bytes / ((double)out->runs * (vb + 16.0)) > kChooseRatio) {
        out->choice = CCQ_CHOOSE_RLE;
        out->rle_runs = out->runs;
    } else if (n_rows >= kChooseMinRows && out->single_runs > 0 && longs > 0 &&
               (double)(n_rows - out->single_runs) * vb / ((double)longs * (vb + 16.0)) > kChooseRatio) {
        out->choice = CCQ_CHOOSE_RLE_INDEX;
        out->rle_runs = longs;
        out->index_points = out->single_runs;
    } else if (n_rows >= kChooseMinRows && w_cut < w_full && w_cut <= 32) {
        out->choice = CCQ_CHOOSE_PLAIN_INDEX;
        out->bit_width = w_cut;
        // centering: codes around the cut range's midpoint (rounded up), so
        // [lo_cut, hi_cut] lies inside [base, base + 2^w)
        const __int128 span = (__int128)out->hi_cut - out->lo_cut;
        const __int128 b = (__int128)out->lo_cut + (span + 1) / 2 - ((__int128)1 << (w_cut - 1));
        out->base = b < (__int128)INT64_MIN ? INT64_MIN : (int64_t)b;
        EncArgs A = {};
        A.values = values;
        A.vtype = value_type;
        A.mode = kModePlainIndex;
        A.n = n_rows;
        A.base = out->base;
        A.w = w_cut;
        int64_t t1;
        if (ccq_status cs = enc_count(A, w, s, &out->index_points, &t1)) return cs;
    } else if (w_full <= 32) {
        out->choice = CCQ_CHOOSE_PLAIN;
        out->bit_width = w_full;
        out->base = out->min_value;
    } else {
        // a range wider than 32 bits has no bit-packed form: runs always do
        out->choice = CCQ_CHOOSE_RLE;
        out->rle_runs = out->runs;
    }
    return ok();
}

ccq_status ccq_plain_to_rle(ccq_context* ctx, const void* values, int32_t value_type, int64_t n_rows, void* ws,
                            size_t ws_bytes, void* stream, void* run_values, int64_t* run_ends, int64_t capacity,
                            int64_t* n_runs) {
    if (!n_runs) return fail(CCQ_E_INVALID, "n_runs is NULL");
    if (ccq_status st = enc_check(ctx, values, value_type, n_rows, ws, ws_bytes)) return st;
    *n_runs = 0;
    if (n_rows == 0) return ok();
    hipStream_t s = (hipStream_t)stream;
    const EncWs w = enc_ws(ws, n_rows);
    EncArgs A = {};
    A.values = values;
    A.vtype = value_type;
    A.out_vtype = value_type;
    A.mode = kModeRle;
    A.n = n_rows;
    int64_t runs, unused;
    if (ccq_status st = enc_count(A, w, s, &runs, &unused)) return st;
    *n_runs = runs;
    if (runs > capacity) return fail(CCQ_E_CAPACITY, "%lld runs, capacity %lld", (long long)runs, (long long)capacity);
    if (!run_values || !run_ends) return fail(CCQ_E_INVALID, "output arrays missing");
    A.run_values = run_values;
    A.run_ends = run_ends;
    launch_write(A, w, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "encode write");
    return ok();
}

ccq_status ccq_plain_to_rle_index(ccq_context* ctx, const void* values, int32_t value_type, int64_t n_rows,
                                  void* ws, size_t ws_bytes, void* stream, void* run_values, int64_t* run_starts,
                                  int64_t* run_ends, int64_t run_capacity, int64_t* idx_positions, void* idx_values,
                                  int64_t idx_capacity, int64_t* n_runs, int64_t* n_points) {
    if (!n_runs || !n_points) return fail(CCQ_E_INVALID, "n_runs / n_points is NULL");
    if (ccq_status st = enc_check(ctx, values, value_type, n_rows, ws, ws_bytes)) return st;
    *n_runs = *n_points = 0;
    if (n_rows == 0) return ok();
    hipStream_t s = (hipStream_t)stream;
    const EncWs w = enc_ws(ws, n_rows);
    EncArgs A = {};
    A.values = values;
    A.vtype = value_type;
    A.out_vtype = value_type;
    A.mode = kModeRleIndex;
    A.n = n_rows;
    int64_t runs, points;
    if (ccq_status st = enc_count(A, w, s, &runs, &points)) return st;
    *n_runs = runs;
    *n_points = points;
    if (runs > run_capacity || points > idx_capacity)
        return fail(CCQ_E_CAPACITY, "%lld runs and %lld points, capacities %lld and %lld", (long long)runs,
                    (long long)points, (long long)run_capacity, (long long)idx_capacity);
    if ((runs && (!run_values || !run_starts || !run_ends)) || (points && (!idx_positions || !idx_values)))
        return fail(CCQ_E_INVALID, "output arrays missing");
    A.run_values = run_values;
    A.run_starts = run_starts;
    A.run_ends = run_ends;
    A.idx_pos = idx_positions;
    A.idx_vals = idx_values;
    launch_write(A, w, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "encode write");
    return ok();
}

ccq_status ccq_plain_to_plain_index(ccq_context* ctx, const void* values, int32_t value_type, int64_t n_rows,
                                    int32_t bit_width, int64_t base, void* ws, size_t ws_bytes, void* stream,
                                    uint32_t* packed, int64_t packed_words, int64_t* idx_positions, void* idx_values,
                                    int64_t idx_capacity, int64_t* n_points) {
    if (!n_points) return fail(CCQ_E_INVALID, "n_points is NULL");
    if (bit_width < 1 || bit_width > 32) return fail(CCQ_E_INVALID, "bit_width must be in 1..32");
    if (ccq_status st = enc_check(ctx, values, value_type, n_rows, ws, ws_bytes)) return st;
    *n_points = 0;
    const int64_t need = (n_rows * (int64_t)bit_width + 31) / 32 + 2;
    if (packed_words < need)
        return fail(CCQ_E_CAPACITY, "packed stream of %lld words, %lld needed", (long long)packed_words,
                    (long long)need);
    if (!packed) return fail(CCQ_E_INVALID, "packed is NULL");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemsetAsync(packed, 0, (size_t)need * 4, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    if (n_rows == 0) return ok();
    const EncWs w = enc_ws(ws, n_rows);
    EncArgs A = {};
    A.values = values;
    A.vtype = value_type;
    A.out_vtype = value_type;
    A.mode = kModePlainIndex;
    A.n = n_rows;
    A.base = base;
    A.w = bit_width;
    int64_t points, unused;
    if (ccq_status st = enc_count(A, w, s, &points, &unused)) return st;
    *n_points = points;
    if (points > idx_capacity)
        return fail(CCQ_E_CAPACITY, "%lld outliers, capacity %lld", (long long)points, (long long)idx_capacity);
    if (points && (!idx_positions || !idx_values)) return fail(CCQ_E_INVALID, "output arrays missing");
    A.idx_pos = idx_positions;
    A.idx_vals = idx_values;
    if (points) launch_write(A, w, s);
    const int64_t lanes = (n_rows + 31) / 32;
    hipLaunchKernelGGL(k_enc_pack, dim3((unsigned)((lanes + kEncThreads - 1) / kEncThreads)), dim3(kEncThreads), 0, s,
                       values, value_type, n_rows, base, bit_width, packed, need);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "encode pack");
    return ok();
}

}  // extern "C"
