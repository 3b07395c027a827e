// lds_gather_probe -- measures the LDS gather ceiling of the device: how many
// 32-bit LDS lookups (one lane each, ds_read_b32) the chip serves per second
// when every lane reads only its own bank, as the round-table kernels do.
//
// Layout, as in the round kernels: 256 rows of 256 bytes; lane l reads
// 4-byte word (l mod 32) of a row (bank l mod 32), or of the row's second
// half (banks 32..63).  Every word holds the byte address of the next lookup
// of the lane that reads it, so each lane walks pointer chains with no VALU
// work between lookups; CHAINS independent chains per lane keep enough
// lookups in flight.  One 1024-thread workgroup per compute unit (the tables
// take 128 KiB).
//
// Reports (one JSON line): lane-gathers per second over the chip (lookups /
// kernel time from HIP events), lane-gathers per shader clock per compute
// unit (s_memtime), the shader clock during the run (s_memtime ticks over
// s_memrealtime's 100 MHz ticks), and the latency of one lookup that depends
// on the one before (one wave per compute unit, one chain; shader clocks per
// lookup, loop included).  A checksum of the chains' end points keeps
// the lookups live.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

namespace {

constexpr int THREADS = 1024;
constexpr int CHAINS = 12;
constexpr uint32_t LDS_BYTES = 131072;  // two 64 KiB regions of 256 rows x 256 B

#define CHECK(x)                                                                         \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) {                                                          \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                      \
            exit(1);                                                                     \
        }                                                                                \
    } while (0)

__global__ __launch_bounds__(THREADS) void k_probe(uint32_t steps, uint32_t *sink,
                                                   unsigned long long *ticks) {
    __shared__ uint32_t lds[LDS_BYTES / 4];
    const uint32_t slot = (threadIdx.x & 31u) << 2;
    // Row x of region g holds, at half h, word slot: the address of row
    // (x * 29 + 71 + h) mod 256, same half and region, same slot.
    for (uint32_t w = threadIdx.x; w < LDS_BYTES / 4; w += blockDim.x) {
        const uint32_t byte = w << 2;
        const uint32_t g = byte >> 16, x = (byte >> 8) & 255u, h = (byte >> 7) & 1u;
        const uint32_t s = byte & 127u;
        const uint32_t nx = (x * 29u + 71u + h) & 255u;
        lds[w] = (g << 16) | (nx << 8) | (h << 7) | s;
    }
    __syncthreads();
    uint32_t a[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; c++) {
        const uint32_t x = (threadIdx.x * 7u + (uint32_t)c * 37u + blockIdx.x) & 255u;
        a[c] = ((uint32_t)(c & 1) << 16) | (x << 8) | ((uint32_t)((c >> 1) & 1) << 7) | slot;
    }
    __syncthreads();
    const unsigned long long t0 = __builtin_amdgcn_s_memtime();
    const unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
    for (uint32_t i = 0; i < steps; i++) {
#pragma unroll
        for (int c = 0; c < CHAINS; c++)
            a[c] = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(lds) +
                                                        a[c]);
    }
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < CHAINS; c++)
        acc ^= a[c];
    __syncthreads();
    const unsigned long long t1 = __builtin_amdgcn_s_memtime();
    const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
    atomicXor(sink, acc);
    if (threadIdx.x == 0) {
        ticks[2 * blockIdx.x] = t1 - t0;
        ticks[2 * blockIdx.x + 1] = r1 - r0;
    }
}

// Latency: one wave per compute unit walking one chain, so every lookup
// waits for the one before; s_memtime ticks per lookup.
__global__ __launch_bounds__(64) void k_latency(uint32_t steps, uint32_t *sink,
                                                unsigned long long *ticks) {
    __shared__ uint32_t lds[LDS_BYTES / 4];
    const uint32_t slot = (threadIdx.x & 31u) << 2;
    for (uint32_t w = threadIdx.x; w < LDS_BYTES / 4; w += blockDim.x) {
        const uint32_t byte = w << 2;
        const uint32_t g = byte >> 16, x = (byte >> 8) & 255u, h = (byte >> 7) & 1u;
        lds[w] = (g << 16) | (((x * 29u + 71u + h) & 255u) << 8) | (h << 7) | (byte & 127u);
    }
    __syncthreads();
    uint32_t a = (((threadIdx.x * 7u + blockIdx.x) & 255u) << 8) | slot;
    const unsigned long long t0 = __builtin_amdgcn_s_memtime();
    for (uint32_t i = 0; i < steps; i++)
        a = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(lds) + a);
    const unsigned long long t1 = __builtin_amdgcn_s_memtime();
    atomicXor(sink, a);
    if (threadIdx.x == 0)
        ticks[blockIdx.x] = t1 - t0;
}

}  // namespace

int main(int argc, char **argv) {
    const int device = argc > 1 ? atoi(argv[1]) : 0;
    const uint32_t steps = argc > 2 ? (uint32_t)atoi(argv[2]) : 8192;
    const int reps = argc > 3 ? atoi(argv[3]) : 5;
    CHECK(hipSetDevice(device));
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, device));
    const int n_cu = prop.multiProcessorCount;
    uint32_t *sink;
    unsigned long long *ticks;
    CHECK(hipMalloc(&sink, sizeof(uint32_t)));
    CHECK(hipMalloc(&ticks, sizeof(unsigned long long) * 2 * n_cu));
    CHECK(hipMemset(sink, 0, sizeof(uint32_t)));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    std::vector<double> ms_all;
    std::vector<double> per_clk_all, ghz_all;
    std::vector<unsigned long long> h(2 * n_cu);
    for (int r = 0; r <= reps; r++) {  // run 0 warms up
        CHECK(hipEventRecord(e0, 0));
        hipLaunchKernelGGL(k_probe, dim3(n_cu), dim3(THREADS), 0, 0, steps, sink, ticks);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(e1, 0));
        CHECK(hipEventSynchronize(e1));
        float ms = 0;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        CHECK(hipMemcpy(h.data(), ticks, sizeof(unsigned long long) * 2 * n_cu,
                        hipMemcpyDeviceToHost));
        if (r == 0)
            continue;
        ms_all.push_back(ms);
        // Per compute unit: lane-gathers of its workgroup over its own clock
        // ticks; shader clock = clock ticks / real-time ticks x 100 MHz.
        double clk = 0, rt = 0;
        for (int g = 0; g < n_cu; g++) {
            clk += (double)h[2 * g];
            rt += (double)h[2 * g + 1];
        }
        const double per_wg = (double)THREADS * CHAINS * steps;
        per_clk_all.push_back(per_wg / (clk / n_cu));
        ghz_all.push_back(clk / rt * 0.1);
    }
    auto med = [](std::vector<double> v) {
        std::sort(v.begin(), v.end());
        return v[v.size() / 2];
    };
    // Latency of one dependent lookup (median over the compute units).
    const uint32_t lat_steps = 4096;
    hipLaunchKernelGGL(k_latency, dim3(n_cu), dim3(64), 0, 0, lat_steps, sink, ticks);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    CHECK(hipMemcpy(h.data(), ticks, sizeof(unsigned long long) * n_cu, hipMemcpyDeviceToHost));
    std::vector<double> lat;
    for (int g = 0; g < n_cu; g++)
        lat.push_back((double)h[g] / lat_steps);
    const double lat_clk = med(lat);
    const double ms = med(ms_all);
    const double total = (double)n_cu * THREADS * CHAINS * steps;
    printf("{\"probe\": \"lds_gather\", \"device\": \"%s\", \"compute_units\": %d, "
           "\"workgroup_threads\": %d, \"chains_per_lane\": %d, \"steps\": %u, \"reps\": %d, "
           "\"kernel_ms_median\": %.4f, \"lane_gathers_per_s\": %.4e, "
           "\"lane_gathers_per_clk_per_cu\": %.3f, \"sclk_ghz\": %.3f, "
           "\"dependent_lookup_clk\": %.1f}\n",
           prop.gcnArchName, n_cu, THREADS, CHAINS, steps, reps, ms, total / (ms * 1e-3),
           med(per_clk_all), med(ghz_all), lat_clk);
    CHECK(hipFree(sink));
    CHECK(hipFree(ticks));
    return 0;
}
