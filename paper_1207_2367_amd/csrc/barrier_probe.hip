// Cost of a barrier across the workgroups of one cooperative launch on the
// MI355X (gfx950): five designs, G resident workgroups of 256 lanes, 2000
// barriers each, with and without 4 KB of data written by every workgroup
// before a barrier and read by its neighbour after it.  Prints one JSON line
// per (design, G, bytes): microseconds per barrier (the slowest workgroup's
// time / barriers).  Every wait is bounded (a timeout sets the error word and
// the run reports it instead of hanging).
//   counter       one arrival counter + one generation word; one agent-scope
//                 release fence before the arrival, one acquire after (the
//                 design of the library's loops)
//   counter_full  the same with a two-way (seq_cst) fence at both points
//   flags         one flag per workgroup, every workgroup polls all flags
//                 (the device loop's first design), two-way fences
//   leader        workgroup 0 polls the flags and releases the others
//                 through one word, two-way fences
//   nofence       the counter without fences: no ordering of the data, not a
//                 valid barrier; the lower bound of the atomic round trips
#include <hip/hip_runtime.h>
#include <cstdio>
#include <vector>

namespace {

constexpr int NT = 256, LINE = 32;   // lanes per workgroup, uint32 words per line
constexpr uint32_t SPINS = 1u << 20;
enum { COUNTER, COUNTER_FULL, FLAGS, LEADER, NOFENCE, NDESIGN };
const char *NAMES[NDESIGN] = {"counter", "counter_full", "flags", "leader", "nofence"};

__device__ __forceinline__ bool wait_for(uint32_t *w, uint32_t e, uint32_t *err)
{
    for (uint32_t k = 0; (int32_t)(__hip_atomic_load(w, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT) - e) < 0; ++k) {
        __builtin_amdgcn_s_sleep(1);
        if (k > SPINS) {
            atomicOr(err, 1u);
            return false;
        }
    }
    return true;
}

template <int D>
__device__ bool barrier(uint32_t *words, uint32_t G, uint32_t *err, uint32_t &epoch)
{
    __shared__ int ok;
    const uint32_t e = ++epoch;
    __syncthreads();
    if (threadIdx.x == 0)
        ok = 1;
    if (D == COUNTER || D == COUNTER_FULL || D == NOFENCE) {
        if (threadIdx.x == 0) {
            uint32_t *cnt = words, *gen = words + LINE;
            if (D == COUNTER)
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            else if (D == COUNTER_FULL)
                __threadfence();
            const uint32_t old = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            if (old == e * G - 1u) {
                if (D == COUNTER)
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __hip_atomic_store(gen, e, D == NOFENCE ? __ATOMIC_RELAXED : __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
            } else if (!wait_for(gen, e, err)) {
                ok = 0;
            }
            if (D == COUNTER)
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            else if (D == COUNTER_FULL)
                __threadfence();
        }
    } else {
        uint32_t *flag = words + 2 * LINE, *rel = words + LINE;
        if (threadIdx.x == 0) {
            __threadfence();
            __hip_atomic_store(&flag[LINE * blockIdx.x], e, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        if (D == FLAGS || blockIdx.x == 0) {
            for (uint32_t f = threadIdx.x; f < G; f += NT)
                if (!wait_for(&flag[LINE * f], e, err)) {
                    ok = 0;
                    break;
                }
        }
        if (D == LEADER) {
            __syncthreads();
            if (blockIdx.x == 0 && threadIdx.x == 0)
                __hip_atomic_store(rel, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else if (blockIdx.x != 0 && threadIdx.x == 0 && !wait_for(rel, e, err))
                ok = 0;
        }
        __threadfence();
    }
    __syncthreads();
    return ok != 0;
}

template <int D>
__global__ __launch_bounds__(NT) void probe(uint32_t *words, uint32_t *err, double *buf,
                                            int iters, int nd, unsigned long long *out)
{
    const uint32_t G = gridDim.x;
    uint32_t epoch = 0;
    double acc = 0.0;
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    int it = 0;
    for (; it < iters; ++it) {
        for (int q = threadIdx.x; q < nd; q += NT)
            buf[(size_t)blockIdx.x * nd + q] = acc + it + q;
        if (!barrier<D>(words, G, err, epoch))
            break;
        const size_t src = (blockIdx.x + 1) % G;
        for (int q = threadIdx.x; q < nd; q += NT)
            acc += buf[src * nd + q];
    }
    const unsigned long long t1 = __builtin_amdgcn_s_memrealtime();
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = t1 - t0;   // 100 MHz ticks
        out[2 * blockIdx.x + 1] = (unsigned long long)it + (acc == -1.0 ? 1 : 0);
    }
}

}  // namespace

#define CK(x)                                                                              \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) {                                                            \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);     \
            return 1;                                                                      \
        }                                                                                  \
    } while (0)

int main()
{
    const int GMAX = 256, NDMAX = 512, ITERS = 2000;
    const void *fn[NDESIGN] = {(const void *)probe<COUNTER>, (const void *)probe<COUNTER_FULL>,
                               (const void *)probe<FLAGS>, (const void *)probe<LEADER>,
                               (const void *)probe<NOFENCE>};
    uint32_t *words, *err;
    double *buf;
    unsigned long long *out;
    const size_t nwords = (size_t)LINE * (GMAX + 2);
    CK(hipMalloc(&words, nwords * 4));
    CK(hipMalloc(&err, 4));
    CK(hipMalloc(&buf, (size_t)GMAX * NDMAX * 8));
    CK(hipMalloc(&out, 2 * GMAX * 8));
    std::vector<unsigned long long> h(2 * GMAX);
    for (int nd : {0, NDMAX})
        for (int G : {16, 32, 64, 128, 256})
            for (int d = 0; d < NDESIGN; ++d) {
                int iters = ITERS;
                CK(hipMemset(words, 0, nwords * 4));
                CK(hipMemset(err, 0, 4));
                void *args[] = {&words, &err, &buf, &iters, &nd, &out};
                CK(hipLaunchCooperativeKernel(fn[d], dim3(G), dim3(NT), args, 0, 0));
                CK(hipDeviceSynchronize());
                uint32_t he = 0;
                CK(hipMemcpy(&he, err, 4, hipMemcpyDeviceToHost));
                CK(hipMemcpy(h.data(), out, 2 * G * 8, hipMemcpyDeviceToHost));
                unsigned long long tmax = 0, done = ~0ull;
                for (int b = 0; b < G; ++b) {
                    tmax = h[2 * b] > tmax ? h[2 * b] : tmax;
                    done = h[2 * b + 1] < done ? h[2 * b + 1] : done;
                }
                std::printf("{\"design\": \"%s\", \"G\": %d, \"bytes_per_wg\": %d, "
                            "\"us_per_barrier\": %.3f, \"barriers\": %llu, \"timeout\": %u}\n",
                            NAMES[d], G, nd * 8, tmax / 100.0 / iters, done, he);
                std::fflush(stdout);
                if (he)
                    return 2;
            }
    return 0;
}
