// Non-template kernels of libccq (clear, finalize, batch clear / finalize,
// validation) and the host launchers that pick a k_fused / k_batch
// instance (instantiated in ccq_inst.hip) for a plan.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "ccq_device.h"

namespace ccq {

// ------------------------------------------------------------------ prepare

__global__ void k_prepare(int64_t* table, int64_t table_len, int32_t* header) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < table_len; i += nt) table[i] = 0;
    if (tid == 0) {
        header[0] = 0;
        header[1] = 0;
    }
}

// ------------------------------------------------------------------ finalize

// Group id g -> key values (last key varies fastest), count and aggregates.
__device__ void write_group(const DevPlan& P, int64_t g, int64_t row, const int64_t* table, int64_t G,
                            int64_t* keys, int64_t* counts, int64_t* aggs) {
    int64_t rem = g;
    for (int k = P.n_keys - 1; k >= 0; --k) {
        const KeyDesc& kd = P.keys[k];
        const int64_t slot = rem % kd.radix;
        rem /= kd.radix;
        const int64_t key = kd.via_lut ? kd.slot_keys[slot] : slot;
        // a dictionary column reports the dictionary entry (the plan checked card <= dict_size)
        keys[row * P.n_keys + k] = kd.dict ? kd.dict[key] : key;
    }
    const int64_t cnt = table[g];
    counts[row] = cnt;
    for (int a = 0; a < P.n_aggs; ++a) {
        const AggDesc& ad = P.aggs[a];
        int64_t v = 0;
        if (ad.kind == kAggCount) {
            v = cnt;
        } else if (cnt > 0) {          // an empty (ungrouped) row reports 0 for every aggregate
            const int64_t c = table[(int64_t)(1 + ad.sum_slot) * G + g];
            v = ad.fin == kFinMin ? min_dec((uint64_t)c) : ad.fin == kFinMax ? max_dec((uint64_t)c) : c;
        }
        aggs[row * P.n_aggs + a] = v;
    }
}

constexpr int64_t kFinPer = (int64_t)kThreads * 16;   // group ids per finalize block

// phase 1: non-empty groups per block of ids
__global__ __launch_bounds__(kThreads) void k_fin_count(const int64_t* table, int64_t G, int64_t* block_cnt) {
    __shared__ int s_part[kWaves];
    const int64_t b0 = (int64_t)blockIdx.x * kFinPer;
    const int64_t b1 = min(b0 + kFinPer, G);
    int c = 0;
    for (int64_t g = b0 + threadIdx.x; g < b1; g += kThreads) c += table[g] > 0;
    for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, 64);
    if (lane_id() == 0) s_part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kWaves; ++w) t += s_part[w];
        block_cnt[blockIdx.x] = t;
    }
}

// phase 2 (one workgroup): exclusive scan of the block counts; total -> n_groups
__global__ __launch_bounds__(kThreads) void k_fin_scan(int64_t* block_cnt, int64_t nb, int64_t* n_groups,
                                                        const int32_t* status_ws, int32_t* status_out) {
    __shared__ int64_t s_tot[kThreads];
    const int64_t per = (nb + kThreads - 1) / kThreads;
    const int64_t a = (int64_t)threadIdx.x * per, b = min(a + per, nb);
    int64_t s = 0;
    for (int64_t i = a; i < b; ++i) s += block_cnt[i];
    s_tot[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int i = 0; i < kThreads; ++i) {
            const int64_t v = s_tot[i];
            s_tot[i] = run;
            run += v;
        }
        *n_groups = run;
        *status_out = *status_ws;
    }
    __syncthreads();
    int64_t run = s_tot[threadIdx.x];
    for (int64_t i = a; i < b; ++i) {
        const int64_t v = block_cnt[i];
        block_cnt[i] = run;
        run += v;
    }
}

// phase 3: write each block's non-empty groups in id order
__global__ __launch_bounds__(kThreads) void k_fin_write(const DevPlan* __restrict__ Pg, const int64_t* table,
                                                         const int64_t* block_off, int64_t* keys, int64_t* counts,
                                                         int64_t* aggs) {
    __shared__ int s_wave[kWaves];
    const DevPlan& P = *Pg;
    const int64_t G = P.n_groups;
    const int64_t b0 = (int64_t)blockIdx.x * kFinPer;
    const int64_t b1 = min(b0 + kFinPer, G);
    int64_t row = block_off[blockIdx.x];
    const int wave = threadIdx.x >> 6;
    for (int64_t base = b0; base < b1; base += kThreads) {
        const int64_t g = base + threadIdx.x;
        const bool ne = g < b1 && table[g] > 0;
        const uint64_t m = wave_ballot(ne);
        if (lane_id() == 0) s_wave[wave] = __builtin_popcountll(m);
        __syncthreads();
        int before = 0, all = 0;
        for (int w = 0; w < kWaves; ++w) {
            if (w < wave) before += s_wave[w];
            all += s_wave[w];
        }
        if (ne) write_group(P, g, row + before + lanes_below(m), table, G, keys, counts, aggs);
        row += all;
        __syncthreads();
    }
}

// ungrouped query: exactly one row, also when nothing qualifies
__global__ void k_fin_single(const DevPlan* __restrict__ Pg, const int64_t* table, int64_t* keys, int64_t* counts,
                             int64_t* aggs, int64_t* n_groups, const int32_t* status_ws, int32_t* status_out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        write_group(*Pg, 0, 0, table, 1, keys, counts, aggs);
        *n_groups = 1;
        *status_out = *status_ws;
    }
}

// Clear each query's region of a batch workspace and the item counters.
__global__ __launch_bounds__(kThreads) void k_batch_clear(const BatchDev* __restrict__ B, unsigned char* ws) {
    if (blockIdx.x == 0 && threadIdx.x < kMaxInstances) B->counters[threadIdx.x] = 0;
    for (int32_t q = blockIdx.x; q < B->n; q += gridDim.x) {
        int64_t* r = (int64_t*)(ws + B->region[q]);
        const int64_t n = B->region_clear[q] / 8;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) r[i] = 0;
    }
}

// Batched finalize: one workgroup per query; grouped queries with more than
// kBatchFinMaxGroups ids are finalized by the multi-block kernels instead.
__global__ __launch_bounds__(kThreads) void k_batch_fin(const BatchDev* __restrict__ B,
                                                         const unsigned char* __restrict__ ws) {
    __shared__ int s_wave[kWaves];
    const int32_t q = blockIdx.x;
    if (q >= B->n) return;      // a grid rounded up for a reusable launch shape
    const DevPlan& P = *B->plans[q];
    const int32_t* status = (const int32_t*)(ws + B->region[q]);
    const int64_t* table = (const int64_t*)(ws + B->region[q] + 256);
    const BatchOut& o = B->outs[q];
    if (P.n_keys == 0) {
        if (threadIdx.x == 0) {
            write_group(P, 0, 0, table, 1, o.keys, o.counts, o.aggs);
            *o.n_groups = 1;
            *o.status = *status;
        }
        return;
    }
    const int64_t G = P.n_groups;
    if (G > kBatchFinMaxGroups) return;
    const int wave = threadIdx.x >> 6;
    int64_t row = 0;
    for (int64_t base = 0; base < G; base += kThreads) {
        const int64_t g = base + threadIdx.x;
        const bool ne = g < G && table[g] > 0;
        const uint64_t m = wave_ballot(ne);
        if (lane_id() == 0) s_wave[wave] = __builtin_popcountll(m);
        __syncthreads();
        int before = 0, all = 0;
        for (int w = 0; w < kWaves; ++w) {
            if (w < wave) before += s_wave[w];
            all += s_wave[w];
        }
        if (ne) write_group(P, g, row + before + lanes_below(m), table, G, o.keys, o.counts, o.aggs);
        row += all;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *o.n_groups = row;
        *o.status = *status;
    }
}

// ------------------------------------------------------------------ validation

__global__ void k_validate_rle(const int64_t* ends, int64_t n, int64_t n_rows, int32_t* flag) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < n; i += nt) {
        const int64_t prev = i == 0 ? 0 : ends[i - 1];
        const int64_t e = ends[i];
        if (e <= prev || (i == n - 1 && e != n_rows)) atomicOr(flag, 1);
    }
}

__global__ void k_validate_idx(const void* pos, int32_t ptype, int64_t n, int64_t n_rows, int32_t* flag) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < n; i += nt) {
        const int64_t p = ld_val(pos, ptype, i);
        const int64_t prev = i == 0 ? -1 : ld_val(pos, ptype, i - 1);
        if (p <= prev || p >= n_rows) atomicOr(flag, 1);
    }
}

// ------------------------------------------------------------------ host launchers

static int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

WsLayout workspace_layout(const DevPlan& p) {
    WsLayout L;
    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t off = 256;
    L.table_off = off;
    off = align(off + sizeof(int64_t) * (size_t)(1 + p.n_sums) * (size_t)p.n_groups);
    L.scan_off = off;
    L.scan_blocks = div_up(p.n_groups, kFinPer);
    off = align(off + sizeof(int64_t) * (size_t)(L.scan_blocks + 1));
    L.total = off;
    return L;
}

// kernel instance for a plan: KMAX bounds the RLE column count, W0 is the
// bit width of the fast row path (0: run mode or generic row mode)
static FusedFn fused_kernel(const DevPlan& p) {
    const bool big = p.fast_big != 0;
    if (p.kmax <= 2) return fused_kernel_k2(kernel_w0(p), big);
    if (p.kmax <= 4) return fused_kernel_k4(kernel_w0(p), big);
    return fused_kernel_k8(kernel_w0(p), big);
}

bool fast_row_width(int w) { return w == 14 || w == 20; }

int fused_grid_limit(const DevPlan& p, int cus) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fused_kernel(p), kThreads,
                                                     p.lds_dyn_bytes) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return per_cu * cus;
}

// Fixed device scratch for callers that cannot allocate: one query's
// workspace (status header, group table, finalize scan), shared by every
// call on the device.  Host code never uses the array's name as an address:
// scratch_address() looks the address up once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(void** out) { return hipGetSymbolAddress(out, HIP_SYMBOL(scratch)); }

// A launch's static plus dynamic LDS must fit the workgroup's LDS: checked
// against the kernel's own attributes before every persistent launch, so a
// plan that asks for too much fails with an error instead of being
// dispatched.  (Attributes and the device limit are looked up once.)
static hipError_t check_lds(const void* fn, size_t dyn) {
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, size_t> stat;
    static std::map<int, size_t> limit;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    size_t st, lim;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = stat.find({dev, fn});
        if (it == stat.end()) {
            hipFuncAttributes a;
            e = hipFuncGetAttributes(&a, fn);
            if (e != hipSuccess) return e;
            it = stat.emplace(std::make_pair(dev, fn), (size_t)a.sharedSizeBytes).first;
        }
        st = it->second;
        auto jt = limit.find(dev);
        if (jt == limit.end()) {
            int v = 0;
            e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
            if (e != hipSuccess) return e;
            jt = limit.emplace(dev, (size_t)v).first;
        }
        lim = jt->second;
    }
    return st + dyn <= lim ? hipSuccess : hipErrorInvalidConfiguration;
}

hipError_t launch_query(const DevPlan& p, const DevPlan* dp, void* ws, hipStream_t stream, int64_t* out_keys,
                        int64_t* out_counts, int64_t* out_aggs, int64_t* out_n_groups, int32_t* out_status,
                        int grid_fused, hipEvent_t ev_begin, hipEvent_t ev_end) {
    if (p.n_tiles > 0) {
        const hipError_t le = check_lds((const void*)fused_kernel(p), (size_t)p.lds_dyn_bytes);
        if (le != hipSuccess) return le;
    }
    const WsLayout L = workspace_layout(p);
    unsigned char* base = (unsigned char*)ws;
    int32_t* header = (int32_t*)base;
    int64_t* table = (int64_t*)(base + L.table_off);
    int64_t* scan = (int64_t*)(base + L.scan_off);
    const int64_t table_len = (int64_t)(1 + p.n_sums) * p.n_groups;

    const int prep_grid = (int)std::min<int64_t>(std::max<int64_t>(div_up(table_len, kThreads), 1), 4096);
    hipLaunchKernelGGL(k_prepare, dim3(prep_grid), dim3(kThreads), 0, stream, table, table_len, header);

    if (ev_begin) {
        hipError_t e = hipEventRecord(ev_begin, stream);
        if (e != hipSuccess) return e;
    }
    if (p.n_tiles > 0) {
        int64_t blocks = std::min<int64_t>(div_up(p.n_tiles, kWaves), grid_fused);
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL(fused_kernel(p), dim3((unsigned)blocks), dim3(kThreads), p.lds_dyn_bytes, stream, dp,
                           table, header, blocks * kWaves);
    }
    if (ev_end) {
        hipError_t e = hipEventRecord(ev_end, stream);
        if (e != hipSuccess) return e;
    }

    if (p.n_keys == 0) {
        hipLaunchKernelGGL(k_fin_single, dim3(1), dim3(64), 0, stream, dp, table, out_keys, out_counts, out_aggs,
                           out_n_groups, header, out_status);
    } else {
        hipLaunchKernelGGL(k_fin_count, dim3((unsigned)L.scan_blocks), dim3(kThreads), 0, stream, table,
                           p.n_groups, scan);
        hipLaunchKernelGGL(k_fin_scan, dim3(1), dim3(kThreads), 0, stream, scan, L.scan_blocks, out_n_groups,
                           header, out_status);
        hipLaunchKernelGGL(k_fin_write, dim3((unsigned)L.scan_blocks), dim3(kThreads), 0, stream, dp, table, scan,
                           out_keys, out_counts, out_aggs);
    }
    return hipGetLastError();
}

static BatchFn batch_kernel(int kmax, int w0, int big) {
    if (kmax <= 2) return batch_kernel_k2(w0, big != 0);
    if (kmax <= 4) return batch_kernel_k4(w0, big != 0);
    return batch_kernel_k8(w0, big != 0);
}

int batch_grid_limit(int kmax, int w0, int big, int lds_bytes, int cus) {
    // occupancy per (instance, LDS bytes), computed once
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int>, int> cache;
    const auto key = std::make_tuple(kmax, w0, big, lds_bytes);
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second * cus;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)batch_kernel(kmax, w0, big), kThreads,
                                                     lds_bytes) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    std::lock_guard<std::mutex> g(mu);
    cache[key] = per_cu;
    return per_cu * cus;
}

hipError_t launch_batch(const BatchDev& host, const BatchDev* dev, const DevPlan* const* plans_host,
                        const DevPlan* const* plans_dev, const int64_t* region, const BatchOut* outs,
                        unsigned char* ws, const int* group_grid, const int* group_lds, const int32_t* big,
                        int32_t n_big, hipStream_t stream, hipEvent_t ev_begin, hipEvent_t ev_end,
                        int32_t fin_grid) {
    for (int g = 0; g < host.n_groups_used; ++g) {
        const BatchGroup& grp = host.groups[g];
        const hipError_t le = check_lds((const void*)batch_kernel(grp.kmax, grp.w0, grp.big), (size_t)group_lds[g]);
        if (le != hipSuccess) return le;
    }
    // fin_grid > 0: a fixed launch shape (for graph replay): every group
    // launches its full persistent grid and the per-query kernels a grid of
    // fin_grid blocks; surplus workgroups exit at once
    const int clear_grid = fin_grid > 0 ? std::min(fin_grid, 4096)
                                        : (int)std::min<int64_t>(std::max<int64_t>(host.n, 1), 4096);
    hipLaunchKernelGGL(k_batch_clear, dim3(clear_grid), dim3(kThreads), 0, stream, dev, ws);
    if (ev_begin) {
        hipError_t e = hipEventRecord(ev_begin, stream);
        if (e != hipSuccess) return e;
    }
    for (int g = 0; g < host.n_groups_used; ++g) {
        const BatchGroup& grp = host.groups[g];
        if (grp.n_items == 0 && fin_grid <= 0) continue;
        const int blocks = fin_grid > 0 ? std::max(1, group_grid[g]) : std::max(1, std::min(group_grid[g], grp.n_items));
        hipLaunchKernelGGL(batch_kernel(grp.kmax, grp.w0, grp.big), dim3(blocks), dim3(kThreads), group_lds[g], stream, dev,
                           g, ws);
    }
    if (ev_end) {
        hipError_t e = hipEventRecord(ev_end, stream);
        if (e != hipSuccess) return e;
    }
    if (host.n > 0)
        hipLaunchKernelGGL(k_batch_fin, dim3(fin_grid > 0 ? fin_grid : host.n), dim3(kThreads), 0, stream, dev, ws);
    for (int i = 0; i < n_big; ++i) {
        // group tables too large for one workgroup: the multi-block finalize
        const int32_t q = big[i];
        const DevPlan& p = *plans_host[q];
        const WsLayout L = workspace_layout(p);
        unsigned char* r = ws + region[q];
        int64_t* table = (int64_t*)(r + L.table_off);
        int64_t* scan = (int64_t*)(r + L.scan_off);
        const int64_t nb = L.scan_blocks;
        hipLaunchKernelGGL(k_fin_count, dim3((unsigned)nb), dim3(kThreads), 0, stream, table, p.n_groups, scan);
        hipLaunchKernelGGL(k_fin_scan, dim3(1), dim3(kThreads), 0, stream, scan, nb, outs[q].n_groups,
                           (const int32_t*)r, outs[q].status);
        hipLaunchKernelGGL(k_fin_write, dim3((unsigned)nb), dim3(kThreads), 0, stream, plans_dev[q], table, scan,
                           outs[q].keys, outs[q].counts, outs[q].aggs);
    }
    return hipGetLastError();
}

hipError_t launch_validate_rle(const int64_t* ends, int64_t n, int64_t n_rows, int32_t* flag, hipStream_t s) {
    const int grid = (int)std::min<int64_t>(std::max<int64_t>(div_up(n, kThreads), 1), 8192);
    hipLaunchKernelGGL(k_validate_rle, dim3(grid), dim3(kThreads), 0, s, ends, n, n_rows, flag);
    return hipGetLastError();
}

hipError_t launch_validate_idx(const void* pos, int32_t ptype, int64_t n, int64_t n_rows, int32_t* flag,
                               hipStream_t s) {
    const int grid = (int)std::min<int64_t>(std::max<int64_t>(div_up(n, kThreads), 1), 8192);
    hipLaunchKernelGGL(k_validate_idx, dim3(grid), dim3(kThreads), 0, s, pos, ptype, n, n_rows, flag);
    return hipGetLastError();
}

}  // namespace ccq
