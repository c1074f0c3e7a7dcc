// noalloc.hip -- the density check for callers that cannot allocate device
// memory: fmmg_check_density_noalloc keeps its per-block partial results in a
// static device array instead of a plan's workspace, calls no allocator, and
// neither synchronises nor copies to the host, so it can run under HIP graph
// capture or in a tight serving loop.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>

#include "launch.h"

namespace fmmg {

namespace {

// Per-block partial results: the smallest flat index of a negative or
// non-finite density in the block's chunk, ~0 if none.  Each GPU the library
// runs on holds one copy until the process ends; every call on that GPU
// shares it (calls that overlap in time on one GPU race).
constexpr int SCRATCH_SLOTS = NOALLOC_SLOTS;
static __device__ __align__(256) unsigned long long scratch[SCRATCH_SLOTS];

constexpr int CHUNK_THREADS = 256;
constexpr int CHUNK = NOALLOC_CHUNK;  // densities per block
constexpr int FINAL_THREADS = 1024;

__device__ __forceinline__ unsigned long long min_u64(unsigned long long a, unsigned long long b) {
    return a < b ? a : b;
}

// One block per chunk of CHUNK densities: every used slot is written, so no
// clearing is needed.
__global__ __launch_bounds__(CHUNK_THREADS) void k_density_partial(const double* __restrict__ rho, int64_t n,
                                                                   unsigned long long* __restrict__ slots) {
    __shared__ unsigned long long wmin[CHUNK_THREADS / 64];
    const int t = threadIdx.x;
    const int64_t base = int64_t(blockIdx.x) * CHUNK;
    unsigned long long m = ~0ull;
#pragma unroll 4
    for (int i = 0; i < CHUNK / CHUNK_THREADS; ++i) {
        const int64_t j = base + int64_t(i) * CHUNK_THREADS + t;  // coalesced
        if (j < n) {
            const double v = rho[j];
            if (!(v >= 0.0) || !(v < __builtin_inf())) m = min_u64(m, (unsigned long long)j);
        }
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) m = min_u64(m, __shfl_xor(m, s));
    if ((t & 63) == 0) wmin[t >> 6] = m;
    __syncthreads();
    if (t == 0) {
        unsigned long long r = wmin[0];
#pragma unroll
        for (int k = 1; k < CHUNK_THREADS / 64; ++k) r = min_u64(r, wmin[k]);
        slots[blockIdx.x] = r;
    }
}

// One block: the smallest of the nb partial results -> out[0] (-1 if none).
__global__ __launch_bounds__(FINAL_THREADS) void k_density_final(const unsigned long long* __restrict__ slots,
                                                                 int nb, int64_t* __restrict__ out) {
    __shared__ unsigned long long wmin[FINAL_THREADS / 64];
    const int t = threadIdx.x;
    unsigned long long m = ~0ull;
    for (int i = t; i < nb; i += FINAL_THREADS) m = min_u64(m, slots[i]);
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) m = min_u64(m, __shfl_xor(m, s));
    if ((t & 63) == 0) wmin[t >> 6] = m;
    __syncthreads();
    if (t == 0) {
        unsigned long long r = wmin[0];
#pragma unroll
        for (int k = 1; k < FINAL_THREADS / 64; ++k) r = min_u64(r, wmin[k]);
        out[0] = r == ~0ull ? int64_t(-1) : int64_t(r);
    }
}

// Device address of `scratch` on each GPU, looked up once per device with
// that device current (the array's name is only a host-side stand-in).
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
unsigned long long* g_scratch_ptr[MAX_DEVICES] = {nullptr};

}  // namespace

hipError_t noalloc_check_density(const double* rho, int64_t n, int64_t* out, hipStream_t st,
                                 std::string* err) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *err = "hipGetDevice";
        return e;
    }
    if (dev < 0 || dev >= MAX_DEVICES) {
        *err = "device index " + std::to_string(dev) + " beyond the supported " + std::to_string(MAX_DEVICES);
        return hipErrorInvalidDevice;
    }
    unsigned long long* slots = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        if (!g_scratch_ptr[dev]) {
            void* p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                *err = "hipGetSymbolAddress(scratch)";
                return e != hipSuccess ? e : hipErrorInvalidSymbol;
            }
            g_scratch_ptr[dev] = static_cast<unsigned long long*>(p);
        }
        slots = g_scratch_ptr[dev];
    }
    const int nb = int((n + CHUNK - 1) / CHUNK);
    if (nb > 0)
        hipLaunchKernelGGL(k_density_partial, dim3(nb), dim3(CHUNK_THREADS), 0, st, rho, n, slots);
    hipLaunchKernelGGL(k_density_final, dim3(1), dim3(FINAL_THREADS), 0, st, slots, nb, out);
    e = hipGetLastError();
    if (e != hipSuccess) *err = "density check launch";
    return e;
}

}  // namespace fmmg
