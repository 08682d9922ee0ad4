// Gather-list copy of frame inputs from pinned host memory to device memory
// in one kernel (the per-frame upload of a serving loop).
#include <hip/hip_runtime.h>

#define FT_KERNELS 1
#include "ft_internal.h"

namespace ft {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kUploadThreads = 256;
constexpr int kUploadVecs = kUploadChunk / (16 * kUploadThreads);   // 16-byte loads per thread
static_assert(kUploadVecs * 16 * kUploadThreads == kUploadChunk, "chunk = whole vector rounds");

__global__ __launch_bounds__(kUploadThreads) void k_upload(UploadArgs a)
{
    const int b = blockIdx.x;
    // segment of this workgroup: the last s with first[s] <= b (empty
    // segments share their successor's first block and are skipped)
    int lo = 0, hi = a.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.first[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const int s = lo;
    const int64_t bytes = a.bytes[s];
    const int64_t beg = (int64_t)(b - a.first[s]) * kUploadChunk;
    const int64_t end = beg + kUploadChunk < bytes ? beg + kUploadChunk : bytes;
    const char *src = a.src[s];
    char *dst = a.dst[s];
    const int64_t nv = (end - beg) >> 4;
    const u32x4 *s4 = reinterpret_cast<const u32x4 *>(src + beg);
    u32x4 *d4 = reinterpret_cast<u32x4 *>(dst + beg);
    u32x4 r[kUploadVecs];
    _Pragma("unroll") for (int k = 0; k < kUploadVecs; ++k)
    {
        const int i = threadIdx.x + k * kUploadThreads;
        if (i < nv) r[k] = s4[i];
    }
    _Pragma("unroll") for (int k = 0; k < kUploadVecs; ++k)
    {
        const int i = threadIdx.x + k * kUploadThreads;
        if (i < nv) d4[i] = r[k];
    }
    if (end == bytes)   // the segment's last chunk: bytes past the last whole vector
        for (int64_t i = beg + (nv << 4) + threadIdx.x; i < end; i += kUploadThreads) dst[i] = src[i];
}

}  // namespace

hipError_t launch_upload(const UploadArgs &a, hipStream_t stream)
{
    if (a.n <= 0 || a.first[a.n] <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_upload, dim3(a.first[a.n]), dim3(kUploadThreads), 0, stream, a);
    return hipGetLastError();
}

}  // namespace ft
