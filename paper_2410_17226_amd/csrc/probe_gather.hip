// Measurement only, not part of libcbfs: the gather ceiling of the pull's arc
// phase.  One pass over a CSR's arcs in CSR order gathers, for every arc k,
// the row state[col[k]] of ROW = 64 * L bytes, with L lanes per arc (64 bytes
// each, four 16-byte loads) and 64 / L arcs per wave step, and ORs it into
// per-lane registers: the arc phase's memory traffic with none of its other
// work (no row ends, scans, early exits, stores).  The time of one pass is the
// floor for a pull round that gathers every arc's set.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

template <int L>
__global__ __launch_bounds__(256) void k_probe_gather(const int32_t *__restrict__ col, int64_t m,
                                                      const ulonglong2 *__restrict__ state,
                                                      unsigned long long *__restrict__ out)
{
    constexpr int AL = 64 / L;
    const int lane = threadIdx.x & 63, h = lane / AL, al = lane % AL;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    unsigned long long a0 = 0, a1 = 0;
    for (int64_t base = wave * AL; base < m; base += nwaves * AL) {
        const int64_t k = base + al;
        if (k < m) {
            const ulonglong2 *p = state + (size_t)col[k] * (4 * L) + h * 4;
            const ulonglong2 x0 = p[0], x1 = p[1], x2 = p[2], x3 = p[3];
            a0 |= x0.x | x1.x | x2.x | x3.x;
            a1 |= x0.y | x1.y | x2.y | x3.y;
        }
    }
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = a0 ^ a1;
}

}  // namespace

// row_bytes in {64, 128, 256}; state holds n rows of row_bytes, every col[k]
// in [0, n); out holds blocks * 256 words.  Returns a hipError_t (0 = launched)
// or -1 for an unsupported row size.
extern "C" int cbfs_probe_gather(int row_bytes, const int32_t *col, int64_t m, const void *state,
                                 unsigned long long *out, int blocks, void *stream)
{
    const ulonglong2 *s = static_cast<const ulonglong2 *>(state);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (row_bytes == 64) hipLaunchKernelGGL(k_probe_gather<1>, dim3(blocks), dim3(256), 0, st, col, m, s, out);
    else if (row_bytes == 128) hipLaunchKernelGGL(k_probe_gather<2>, dim3(blocks), dim3(256), 0, st, col, m, s, out);
    else if (row_bytes == 256) hipLaunchKernelGGL(k_probe_gather<4>, dim3(blocks), dim3(256), 0, st, col, m, s, out);
    else return -1;
    return (int)hipGetLastError();
}
