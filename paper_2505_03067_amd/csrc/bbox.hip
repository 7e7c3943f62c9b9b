// Bounding box of all tumour cells plus a margin (paper Sec. 2.3).
//
// One streaming pass over the int32 cell-id lattice.  Each thread keeps the
// extremes of the voxels it visits; each block reduces them (cross-lane shuffles,
// then LDS) to one partial, and a second one-block kernel folds the partials.  No
// atomics: thousands of waves updating the same six words would serialise on one
// cache line.
#include <map>
#include <mutex>
#include <utility>

#include "common.h"

namespace mpm {

__device__ inline int wave_min(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ inline int wave_max(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

constexpr int kBboxBlocks = 1024;   // blocks of the streaming pass (one partial each)

// Scratch of mpm_bbox_from_cells_noalloc, one copy per device for the life of the
// process: the six folded extremes (words 0..5, padded to 8) and the six extremes of
// each block of the streaming pass.  The kernels write every word they read, so no
// call needs it cleared.  In host code this name is only a handle: kernels are given
// the device address that hipGetSymbolAddress returns for the current device.
constexpr int kBboxScratchWords = 8 + 6 * kBboxBlocks;
static __device__ __align__(256) int scratch[kBboxScratchWords];

// Extremes of one block: wave reduction, then the block's waves through LDS.  Thread
// 0 returns them in mn/mx.
__device__ inline void block_extremes(int (&mn)[3], int (&mx)[3]) {
    __shared__ int sh[4][6];
    const int wave = threadIdx.x >> 6;
    for (int d = 0; d < 3; ++d) {
        mn[d] = wave_min(mn[d]);
        mx[d] = wave_max(mx[d]);
    }
    if ((threadIdx.x & 63) == 0)
        for (int d = 0; d < 3; ++d) {
            sh[wave][d] = mn[d];
            sh[wave][3 + d] = mx[d];
        }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
            for (int d = 0; d < 3; ++d) {
                mn[d] = min(mn[d], sh[w][d]);
                mx[d] = max(mx[d], sh[w][3 + d]);
            }
}

__device__ inline void store_partial(int* part, const int (&mn)[3], const int (&mx)[3]) {
    if (threadIdx.x == 0)
        for (int d = 0; d < 3; ++d) {
            part[blockIdx.x * 6 + d] = mn[d];
            part[blockIdx.x * 6 + 3 + d] = mx[d];
        }
}

// Vector path: nx % 4 == 0, so the four voxels of an int4 share one row.  Writes the
// block's extremes to part[block][0..5] (min x, y, z; max x, y, z; INT_MAX / -1 if the
// block saw no cell voxel).
__global__ __launch_bounds__(256) void k_bbox_vec4(const int4* __restrict__ cell, long long nquad,
                                                   int nx, int ny, int* __restrict__ part) {
    int mn[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff};
    int mx[3] = {-1, -1, -1};
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nquad; q += stride) {
        int4 c = cell[q];
        int any = (c.x > 0) | (c.y > 0) | (c.z > 0) | (c.w > 0);
        if (any) {
            long long i = q * 4;
            long long row = i / nx;
            int x = (int)(i - row * nx);
            int z = (int)(row / ny);
            int y = (int)(row - (long long)z * ny);
            int first = c.x > 0 ? 0 : (c.y > 0 ? 1 : (c.z > 0 ? 2 : 3));
            int last = c.w > 0 ? 3 : (c.z > 0 ? 2 : (c.y > 0 ? 1 : 0));
            mn[0] = min(mn[0], x + first);
            mx[0] = max(mx[0], x + last);
            mn[1] = min(mn[1], y);
            mx[1] = max(mx[1], y);
            mn[2] = min(mn[2], z);
            mx[2] = max(mx[2], z);
        }
    }
    block_extremes(mn, mx);
    store_partial(part, mn, mx);
}

// Scalar path for any nx (same output).
__global__ __launch_bounds__(256) void k_bbox_scalar(const int* __restrict__ cell, long long n,
                                                     int nx, int ny, int* __restrict__ part) {
    int mn[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff};
    int mx[3] = {-1, -1, -1};
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (cell[i] > 0) {
            long long row = i / nx;
            int x = (int)(i - row * nx);
            int z = (int)(row / ny);
            int y = (int)(row - (long long)z * ny);
            mn[0] = min(mn[0], x); mx[0] = max(mx[0], x);
            mn[1] = min(mn[1], y); mx[1] = max(mx[1], y);
            mn[2] = min(mn[2], z); mx[2] = max(mx[2], z);
        }
    }
    block_extremes(mn, mx);
    store_partial(part, mn, mx);
}

// One block folds the per-block partials into ext[0..5].  Integer min/max does not
// depend on the order, so the result is exact.
__global__ __launch_bounds__(256) void k_bbox_final(const int* __restrict__ part, int nparts,
                                                    int* __restrict__ ext) {
    int mn[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff};
    int mx[3] = {-1, -1, -1};
    for (int b = threadIdx.x; b < nparts; b += blockDim.x)
        for (int d = 0; d < 3; ++d) {
            mn[d] = min(mn[d], part[b * 6 + d]);
            mx[d] = max(mx[d], part[b * 6 + 3 + d]);
        }
    block_extremes(mn, mx);
    if (threadIdx.x == 0)
        for (int d = 0; d < 3; ++d) {
            ext[d] = mn[d];
            ext[3 + d] = mx[d];
        }
}

// Both passes of the box search into ext[0..5] (ext + 8 holds the per-block partials).
static void launch_bbox(const int32_t* cell_id, const int32_t* dims, int* ext, hipStream_t st) {
    const long long n = (long long)dims[0] * dims[1] * dims[2];
    int* part = ext + 8;
    if (dims[0] % 4 == 0 && ((uintptr_t)cell_id % 16) == 0) {
        k_bbox_vec4<<<kBboxBlocks, 256, 0, st>>>((const int4*)cell_id, n / 4, dims[0], dims[1], part);
    } else {
        k_bbox_scalar<<<kBboxBlocks, 256, 0, st>>>(cell_id, n, dims[0], dims[1], part);
    }
    k_bbox_final<<<1, 256, 0, st>>>(part, kBboxBlocks, ext);
}

// The box from the six extremes read back to the host (max x < 0: no cell voxel).
static int box_from_extremes(const int* ext, const int32_t* dims, int32_t margin, int32_t* lo, int32_t* hi,
                             const char* who) {
    if (ext[3] < 0) {
        set_error(std::string(who) + ": no voxel with a positive cell id");
        return MPM_EEMPTY;
    }
    for (int d = 0; d < 3; ++d) {
        int a = ext[d] - margin;
        int b = ext[3 + d] + margin + 1;
        lo[d] = a < 0 ? 0 : a;
        hi[d] = b > dims[d] ? dims[d] : b;
    }
    return MPM_OK;
}

static int check_bbox_args(const int32_t* cell_id, const int32_t* dims, int32_t margin, const int32_t* lo,
                           const int32_t* hi, const char* who) {
    if (!cell_id || !dims || !lo || !hi) {
        set_error(std::string(who) + ": null pointer");
        return MPM_EINVAL;
    }
    if (dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0 || margin < 0) {
        set_error(std::string(who) + ": dims must be positive and margin non-negative");
        return MPM_EINVAL;
    }
    return MPM_OK;
}

}  // namespace mpm

using namespace mpm;

extern "C" int32_t mpm_bbox_from_cells_noalloc(const int32_t* cell_id, const int32_t* dims, int32_t margin,
                                               int32_t* lo, int32_t* hi, void* stream) {
    const char* who = "mpm_bbox_from_cells_noalloc";
    int rc = check_bbox_args(cell_id, dims, margin, lo, hi, who);
    if (rc != MPM_OK) return rc;
    // device address of this device's copy of the scratch array, looked up once per
    // device (the array's name is not a device address in host code)
    static std::mutex mu;
    static std::map<int, int*> addr;
    int dev = 0;
    MPM_HIP(hipGetDevice(&dev));
    int* ext = nullptr;
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = addr.find(dev);
        if (it == addr.end()) {
            void* p = nullptr;
            hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, who);
            it = addr.emplace(dev, (int*)p).first;
        }
        ext = it->second;
    }
    hipStream_t st = (hipStream_t)stream;
    launch_bbox(cell_id, dims, ext, st);
    int host[6];
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(host, ext, sizeof(host), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, who);
    return box_from_extremes(host, dims, margin, lo, hi, who);
}

extern "C" int32_t mpm_bbox_from_cells(const int32_t* cell_id, const int32_t* dims, int32_t margin,
                                       int32_t* lo, int32_t* hi, void* stream) {
    int rc0 = check_bbox_args(cell_id, dims, margin, lo, hi, "mpm_bbox_from_cells");
    if (rc0 != MPM_OK) return rc0;
    hipStream_t st = (hipStream_t)stream;
    // six device words and their pinned host copy, allocated once per device and kept
    // until the process ends (a box recomputed every step then allocates nothing);
    // calls from several threads take turns
    static std::mutex mu;
    static std::map<int, std::pair<int*, int*>> bufs;
    std::lock_guard<std::mutex> lock(mu);
    int dev = 0;
    MPM_HIP(hipGetDevice(&dev));
    auto it = bufs.find(dev);
    if (it == bufs.end()) {
        int* ext = nullptr;
        int* host = nullptr;
        MPM_HIP(hipMalloc(&ext, (8 + 6 * kBboxBlocks) * sizeof(int)));
        hipError_t e = hipHostMalloc((void**)&host, 8 * sizeof(int), hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipFree(ext);
            return hip_fail(e, "hipHostMalloc");
        }
        it = bufs.emplace(dev, std::make_pair(ext, host)).first;
    }
    int* ext = it->second.first;
    int* host = it->second.second;
    launch_bbox(cell_id, dims, ext, st);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(host, ext, 6 * sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "mpm_bbox_from_cells");
    return box_from_extremes(host, dims, margin, lo, hi, "mpm_bbox_from_cells");
}
