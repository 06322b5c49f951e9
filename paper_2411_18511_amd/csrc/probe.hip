// Streaming bandwidth probe: the HBM rate this device reaches for a given
// read/write mix, measured with the same access instructions as the operator
// kernels (16-byte non-temporal loads and stores, XCD-aware block order).  It
// is the ceiling the memory-bound kernels are compared with.
#include "api_util.h"
#include "hrd.h"

namespace hrd {
namespace {

// dst element i = sum over j < k of source element (i, j).  Layout 0: the
// source is k separate streams of nw elements (element (i, j) at j nw + i), as
// a kernel reading k planes stored one array per plane.  Layout 1: 64-element
// tiles, source element (i, j) at (i / 64) 64 k + j 64 + i % 64, so a wave reads
// one contiguous 1 KiB x k stretch per tile (the 64-site tile layout).
template <int LAYOUT>
__global__ __launch_bounds__(256) void stream_probe_kernel(const vd2 *__restrict__ src, vd2 *__restrict__ dst,
                                                           long nw, int k)
{
    const long lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const long i = lb * 256 + threadIdx.x;
    if (i >= nw) return;
    vd2 acc = vd2{0.0, 0.0};
    if constexpr (LAYOUT == 0) {
        for (int j = 0; j < k; j++) acc += __builtin_nontemporal_load(src + (long)j * nw + i);
    } else {
        const vd2 *t = src + (i >> 6) * 64 * (long)k + (i & 63);
        for (int j = 0; j < k; j++) acc += __builtin_nontemporal_load(t + j * 64);
    }
    __builtin_nontemporal_store(acc, dst + i);
}

}  // namespace
}  // namespace hrd

using namespace hrd;

hrd_status hrd_stream_probe(const void *src, size_t read_bytes, void *dst, size_t write_bytes, int tiled,
                            void *stream)
{
    if (!src || !dst) return fail(HRD_EINVAL, "stream_probe: null buffer");
    if (write_bytes == 0 || write_bytes % 16 != 0)
        return fail(HRD_EINVAL, "stream_probe: write_bytes must be a positive multiple of 16");
    if (read_bytes % write_bytes != 0 || read_bytes / write_bytes < 1 || read_bytes / write_bytes > 64)
        return fail(HRD_EINVAL, "stream_probe: read_bytes must be k * write_bytes with 1 <= k <= 64");
    if (tiled != 0 && tiled != 1) return fail(HRD_EINVAL, "stream_probe: tiled must be 0 or 1");
    if (tiled && write_bytes % 1024 != 0)
        return fail(HRD_EINVAL, "stream_probe: the tiled layout needs write_bytes to be a multiple of 1024");
    if (overlap(src, read_bytes, dst, write_bytes)) return fail(HRD_EALIAS, "stream_probe: src and dst overlap");
    const long nw = (long)(write_bytes / 16);
    const int k = (int)(read_bytes / write_bytes);
    const long nblk = (nw + 255) / 256;
    if (nblk > 0x7fffffffL) return fail(HRD_EINVAL, "stream_probe: too many elements for one launch");
    hipStream_t st = (hipStream_t)stream;
    if (tiled)
        hipLaunchKernelGGL(stream_probe_kernel<1>, dim3((unsigned)nblk), dim3(256), 0, st, (const vd2 *)src,
                           (vd2 *)dst, nw, k);
    else
        hipLaunchKernelGGL(stream_probe_kernel<0>, dim3((unsigned)nblk), dim3(256), 0, st, (const vd2 *)src,
                           (vd2 *)dst, nw, k);
    return check_hip(hipGetLastError(), "stream_probe launch");
}
