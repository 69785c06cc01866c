// Allocation-free advance of libfskmc (fskmc_advance_noalloc): the static
// device scratch it works in, the per-device lookup of that array's address,
// and the small kernels that fill it (rate table from kernel arguments, block
// lists of the built-in colour maps) and read the results out of it.  The
// sweep itself is the one-launch-per-window kernel of fskmc_kernels.hip.
#include "fskmc_internal.h"

#include <algorithm>
#include <mutex>

namespace fskmc {

// Allocation-free advance.  Its working memory (rate table, block lists,
// counter records) is this file-scope array; each GPU holds its own copy for
// the life of the process.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): it uses the
// device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint8_t scratch[kNoallocBytes];

hipError_t noalloc_scratch(int device, uint8_t** out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static uint8_t* addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices || !out)
        return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess)
            return e;
        if ((e = hipSetDevice(device)) != hipSuccess)
            return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t r = hipSetDevice(prev);
        if (e != hipSuccess)
            return e;
        if (r != hipSuccess)
            return r;
        addr[device] = static_cast<uint8_t*>(p);
    }
    *out = addr[device];
    return hipSuccess;
}

// Up to 480 doubles per launch travel in the kernel arguments (3840 bytes).
struct F64Chunk {
    double v[480];
};

__global__ void k_put_f64(double* dst, F64Chunk c, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        dst[i] = c.v[i];
}

hipError_t launch_put_f64(double* dst, const double* host, int n, hipStream_t s)
{
    for (int i0 = 0; i0 < n; i0 += 480) {
        const int k = std::min(480, n - i0);
        F64Chunk c;
        for (int i = 0; i < k; ++i)
            c.v[i] = host[i0 + i];
        hipLaunchKernelGGL(k_put_f64, dim3((k + 255) / 256), dim3(256), 0, s, dst + i0, c, k);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// Position of block m = (bi, bj) in the colour-grouped list of a built-in map:
// the blocks of its colour in earlier rows (rows of the matching parity hold
// ceil or floor of NBX/2 of them) plus those left of it in its row (every
// second column, bi/2 of them either way).
__global__ void k_builtin_blocks(int32_t* out, int NBX, int NBY, int K, int4 off)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= NBX * NBY)
        return;
    const int bi = m % NBX, bj = m / NBX;
    const int even = (NBX + 1) / 2, odd = NBX / 2; // columns of even / odd index in a row
    int c, rank;
    if (K == 2) {
        c = (bi + bj) & 1;
        // rows j < bj whose blocks of colour c sit in even columns: j = c mod 2
        const int rows_even = c == 0 ? (bj + 1) / 2 : bj / 2;
        rank = rows_even * even + (bj - rows_even) * odd + bi / 2;
    } else {
        c = (bi & 1) + 2 * (bj & 1);
        rank = (bj / 2) * ((bi & 1) ? odd : even) + bi / 2;
    }
    const int base = c == 0 ? off.x : c == 1 ? off.y : c == 2 ? off.z : off.w;
    out[base + rank] = m;
}

hipError_t launch_builtin_blocks(int32_t* out, int NBX, int NBY, int n_colours, const int32_t off[4], hipStream_t s)
{
    const int nb = NBX * NBY;
    if (nb <= 0 || (n_colours != 2 && n_colours != 4))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_builtin_blocks, dim3((nb + 255) / 256), dim3(256), 0, s, out, NBX, NBY, n_colours,
                       make_int4(off[0], off[1], off[2], off[3]));
    return hipGetLastError();
}

// One workgroup: W of every block, and the events summed over the blocks.
__global__ __launch_bounds__(1024) void k_noalloc_outputs(const BlockCount* __restrict__ cnt, int nb, uint32_t* W,
                                                          unsigned long long* events)
{
    __shared__ unsigned long long part[16];
    unsigned long long sum = 0;
    for (int m = threadIdx.x; m < nb; m += 1024) {
        if (W)
            W[m] = cnt[m].W;
        sum += cnt[m].events;
    }
    for (int o = 32; o > 0; o >>= 1)
        sum += __shfl_down(sum, o);
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0 && events) {
        unsigned long long t = 0;
        for (int i = 0; i < 16; ++i)
            t += part[i];
        *events = t;
    }
}

hipError_t launch_noalloc_outputs(const BlockCount* cnt, int nb, uint32_t* W, unsigned long long* events,
                                  hipStream_t s)
{
    hipLaunchKernelGGL(k_noalloc_outputs, dim3(1), dim3(1024), 0, s, cnt, nb, W, events);
    return hipGetLastError();
}

}  // namespace fskmc
