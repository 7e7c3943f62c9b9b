// Streaming probes of the memory system: the practical bandwidth ceiling of a kernel
// that streams through HBM, measured with the launch shape of the solver kernels
// (256-thread blocks, 16-byte accesses, grid-stride loops).  The solver kernels are
// judged against these rates as well as against the 8 TB/s datasheet peak.
#include "common.h"

namespace mpm {

typedef float v4f __attribute__((ext_vector_type(4)));

// Sum of a v4f array: per-block partial sums into part[block] (keeps the loads live).
// Four independent 16-byte loads in flight per thread and iteration.
template <bool NT>
__global__ __launch_bounds__(256) void k_probe_read(const v4f* __restrict__ a, long long n4,
                                                    float* __restrict__ part) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    v4f s = v4f{0.f, 0.f, 0.f, 0.f};
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        v4f v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = NT ? __builtin_nontemporal_load(a + i + u * stride) : a[i + u * stride];
#pragma unroll
        for (int u = 0; u < 4; ++u) s += v[u];
    }
    for (; i < n4; i += stride) {
        s += a[i];
    }
    float t = (s.x + s.y) + (s.z + s.w);
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    __shared__ float sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// c = a (NT: nontemporal stores), or c = a + s b (TRIAD).
template <bool TRIAD, bool NT>
__global__ __launch_bounds__(256) void k_probe_stream(const v4f* __restrict__ a, const v4f* __restrict__ b,
                                                      v4f* __restrict__ c, float s, long long n4) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + stride < n4; i += 2 * stride) {
        v4f x0 = a[i], x1 = a[i + stride];
        if (TRIAD) {
            const v4f y0 = b[i], y1 = b[i + stride];
            x0 = x0 + s * y0;
            x1 = x1 + s * y1;
        }
        if (NT) {
            __builtin_nontemporal_store(x0, c + i);
            __builtin_nontemporal_store(x1, c + i + stride);
        } else {
            c[i] = x0;
            c[i + stride] = x1;
        }
    }
    for (; i < n4; i += stride) {
        v4f x = a[i];
        if (TRIAD) {
            const v4f y = b[i];
            x = x + s * y;
        }
        c[i] = x;
    }
}

static int launch_probe(int kind, bool nt, const void* a, const void* b, void* c, long long n4, int blocks,
                        hipStream_t st) {
    const v4f* A = (const v4f*)a;
    const v4f* B = (const v4f*)b;
    v4f* C = (v4f*)c;
    switch (kind) {
        case MPM_PROBE_READ:
            if (nt) k_probe_read<true><<<blocks, 256, 0, st>>>(A, n4, (float*)c);
            else k_probe_read<false><<<blocks, 256, 0, st>>>(A, n4, (float*)c);
            break;
        case MPM_PROBE_COPY:
            if (nt) k_probe_stream<false, true><<<blocks, 256, 0, st>>>(A, nullptr, C, 0.f, n4);
            else k_probe_stream<false, false><<<blocks, 256, 0, st>>>(A, nullptr, C, 0.f, n4);
            break;
        default:
            if (nt) k_probe_stream<true, true><<<blocks, 256, 0, st>>>(A, B, C, 3.f, n4);
            else k_probe_stream<true, false><<<blocks, 256, 0, st>>>(A, B, C, 3.f, n4);
            break;
    }
    MPM_HIP(hipGetLastError());
    return MPM_OK;
}

}  // namespace mpm

using namespace mpm;

extern "C" int32_t mpm_hbm_probe(int32_t kind, const void* a, const void* b, void* c, int64_t bytes, int32_t blocks,
                                 int32_t repeat, void* stream, double* ms) {
    const int base = kind & 0xff;
    const bool nt = (kind & MPM_PROBE_NONTEMPORAL) != 0;
    if (!a || !c || !ms || bytes <= 0 || bytes % 16 || blocks < 1 || blocks > (1 << 20) || repeat < 1 ||
        repeat > 1000 || base < MPM_PROBE_READ || base > MPM_PROBE_TRIAD || (kind & ~(0xff | MPM_PROBE_NONTEMPORAL)) ||
        (base == MPM_PROBE_TRIAD && !b) || (((uintptr_t)a | (uintptr_t)c | (uintptr_t)b) % 16)) {
        set_error("mpm_hbm_probe: bad arguments");
        return MPM_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    const long long n4 = bytes / 16;
    // one untimed launch, then 'repeat' launches between two events
    int rc = launch_probe(base, nt, a, b, c, n4, blocks, st);
    if (rc != MPM_OK) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    MPM_HIP(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < repeat && e == hipSuccess && rc == MPM_OK; ++r) rc = launch_probe(base, nt, a, b, c, n4, blocks, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc != MPM_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "mpm_hbm_probe");
    *ms = (double)t / repeat;
    return MPM_OK;
}
