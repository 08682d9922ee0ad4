// Local-map edits of several maps in two launches: every move (a removed slot
// below the new count taking a surviving tail point) of every edit, then
// every append.  Moves never overlap within one map (holes lie below the new
// count, sources at or above it), and an append may land on a source slot, so
// the appends wait for the moves (stream order).
#include <hip/hip_runtime.h>

#define FT_KERNELS 1
#include "ft_internal.h"

namespace ft {

namespace {

constexpr int kThreads = 256;

// Kernel argument: the edits' descriptors and one list (moves or appends).
struct ManyArgs {
    const FT_G MapEditDesc *descs;
    const FT_G int32_t *list;
    int n;
};

// One point's 64-byte record (position, normal, distance bounds, descriptor).
__device__ __forceinline__ void copy_point(const MapEditDesc &d, int to, const FT_G float *pos,
                                           const FT_G float *normal, const FT_G float *dmin, const FT_G float *dmax,
                                           const FT_G uint8_t *desc, int from)
{
    float p[3], nr[3];
    _Pragma("unroll") for (int c = 0; c < 3; ++c)
    {
        p[c] = pos[3 * from + c];
        nr[c] = normal[3 * from + c];
    }
    const float d0 = dmin[from], d1 = dmax[from];
    const uint4 q0 = reinterpret_cast<const FT_G uint4 *>(desc + 32 * (size_t)from)[0];
    const uint4 q1 = reinterpret_cast<const FT_G uint4 *>(desc + 32 * (size_t)from)[1];
    _Pragma("unroll") for (int c = 0; c < 3; ++c)
    {
        d.pos[3 * to + c] = p[c];
        d.normal[3 * to + c] = nr[c];
    }
    d.dmin[to] = d0;
    d.dmax[to] = d1;
    reinterpret_cast<FT_G uint4 *>(d.desc + 32 * (size_t)to)[0] = q0;
    reinterpret_cast<FT_G uint4 *>(d.desc + 32 * (size_t)to)[1] = q1;
}

__global__ __launch_bounds__(kThreads) void k_map_move_many(ManyArgs a)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= a.n) return;
    const MapEditDesc d = a.descs[a.list[3 * i]];
    copy_point(d, a.list[3 * i + 1], d.pos, d.normal, d.dmin, d.dmax, d.desc, a.list[3 * i + 2]);
}

__global__ __launch_bounds__(kThreads) void k_map_append_many(ManyArgs a)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= a.n) return;
    const MapEditDesc d = a.descs[a.list[2 * i]];
    const int j = a.list[2 * i + 1];
    copy_point(d, d.n1 + j, d.ipos, d.inormal, d.idmin, d.idmax, d.idesc, j);
}

}  // namespace

hipError_t launch_map_edit_many(const MapEditDesc *descs, const int32_t *moves, int n_moves, const int32_t *apps,
                                int n_apps, hipStream_t s)
{
    if (n_moves > 0) {
        ManyArgs a{};
        a.descs = (const FT_G MapEditDesc *)descs;   // global memory: the context's staging
        a.list = (const FT_G int32_t *)moves;
        a.n = n_moves;
        hipLaunchKernelGGL(k_map_move_many, dim3((n_moves + kThreads - 1) / kThreads), dim3(kThreads), 0, s, a);
    }
    if (n_apps > 0) {
        ManyArgs a{};
        a.descs = (const FT_G MapEditDesc *)descs;
        a.list = (const FT_G int32_t *)apps;
        a.n = n_apps;
        hipLaunchKernelGGL(k_map_append_many, dim3((n_apps + kThreads - 1) / kThreads), dim3(kThreads), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace ft
