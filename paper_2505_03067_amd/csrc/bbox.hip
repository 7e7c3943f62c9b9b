// Bounding box of all tumour cells plus a margin (paper Sec. 2.3).
//
// One streaming pass over the int32 cell-id lattice.  Each thread keeps the
// extremes of the voxels it visits, a wave64 reduces them with cross-lane
// shuffles, and one integer atomic per wave and bound folds them into six device
// words.  Integer min/max is order independent, so the result is exact.
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

// ext[0..2] = min x, y, z (init INT_MAX); ext[3..5] = max x, y, z (init -1).
__global__ __launch_bounds__(256) void k_bbox_init(int* ext) {
    if (threadIdx.x < 3) ext[threadIdx.x] = 0x7fffffff;
    else if (threadIdx.x < 6) ext[threadIdx.x] = -1;
}

// Vector path: nx % 4 == 0, so the four voxels of an int4 share one row.
__global__ __launch_bounds__(256) void k_bbox_vec4(const int4* __restrict__ cell, long long nquad,
                                                   int nx, int ny, int* ext) {
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
    for (int d = 0; d < 3; ++d) {
        int a = wave_min(mn[d]);
        int b = wave_max(mx[d]);
        if ((threadIdx.x & 63) == 0) {
            if (b >= 0) {
                atomicMin(ext + d, a);
                atomicMax(ext + 3 + d, b);
            }
        }
    }
}

// Scalar path for any nx.
__global__ __launch_bounds__(256) void k_bbox_scalar(const int* __restrict__ cell, long long n,
                                                     int nx, int ny, int* ext) {
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
    for (int d = 0; d < 3; ++d) {
        int a = wave_min(mn[d]);
        int b = wave_max(mx[d]);
        if ((threadIdx.x & 63) == 0 && b >= 0) {
            atomicMin(ext + d, a);
            atomicMax(ext + 3 + d, b);
        }
    }
}

}  // namespace mpm

using namespace mpm;

extern "C" int32_t mpm_bbox_from_cells(const int32_t* cell_id, const int32_t* dims, int32_t margin,
                                       int32_t* lo, int32_t* hi, void* stream) {
    if (!cell_id || !dims || !lo || !hi) {
        set_error("mpm_bbox_from_cells: null pointer");
        return MPM_EINVAL;
    }
    if (dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0 || margin < 0) {
        set_error("mpm_bbox_from_cells: dims must be positive and margin non-negative");
        return MPM_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    const long long n = (long long)dims[0] * dims[1] * dims[2];
    int* ext = nullptr;
    int* host = nullptr;
    MPM_HIP(hipMalloc(&ext, 8 * sizeof(int)));
    hipError_t e = hipHostMalloc((void**)&host, 8 * sizeof(int), hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipFree(ext);
        return hip_fail(e, "hipHostMalloc");
    }
    k_bbox_init<<<1, 64, 0, st>>>(ext);
    const int grid = 2048;
    if (dims[0] % 4 == 0 && ((uintptr_t)cell_id % 16) == 0) {
        k_bbox_vec4<<<grid, 256, 0, st>>>((const int4*)cell_id, n / 4, dims[0], dims[1], ext);
    } else {
        k_bbox_scalar<<<grid, 256, 0, st>>>(cell_id, n, dims[0], dims[1], ext);
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(host, ext, 6 * sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    int r = MPM_OK;
    if (e != hipSuccess) {
        r = hip_fail(e, "mpm_bbox_from_cells");
    } else if (host[3] < 0) {
        set_error("mpm_bbox_from_cells: no voxel with a positive cell id");
        r = MPM_EEMPTY;
    } else {
        for (int d = 0; d < 3; ++d) {
            int a = host[d] - margin;
            int b = host[3 + d] + margin + 1;
            lo[d] = a < 0 ? 0 : a;
            hi[d] = b > dims[d] ? dims[d] : b;
        }
    }
    (void)hipFree(ext);
    (void)hipHostFree(host);
    return r;
}
