// Hand-off latency between compute units, the cost of one neighbour hand-off
// in the persistent sweeps: two workgroups (one active lane each) pass a
// counter back and forth through two 32-bit words 128 bytes apart, each side
// storing with one cache policy and polling with another, for workgroup pairs
// on the same XCD and on two different ones (workgroups are dispatched
// round-robin over the XCDs; each reports its XCC_ID hardware register).
// Policies are the cache bits of the buffer instructions: 0 none, 1 sc0
// (workgroup scope), 16 sc1 (device scope), 17 sc0 sc1 (system scope).
// Every wait is bounded (2e6 polls or 2 s of the 100 MHz wall clock), and a
// pair whose reader never sees the writer's value reports a time-out.
//
//   hipcc --offload-arch=gfx950 -O3 -o handoff_probe tests/native/handoff_probe.hip && ./handoff_probe
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdint.h>

__device__ __forceinline__ uint64_t wclk() { return __builtin_amdgcn_s_memrealtime(); } // 100 MHz

__device__ __forceinline__ uint32_t ld(__amdgpu_buffer_rsrc_t r, int off, int pol)
{
    switch (pol) {
    case 0: return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
    case 1: return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 1);
    case 16: return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 16);
    default: return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 17);
    }
}
__device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, int off, uint32_t v, int pol)
{
    switch (pol) {
    case 0: __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, 0); break;
    case 1: __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, 1); break;
    case 16: __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, 16); break;
    default: __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, 17); break;
    }
}

// buf: 64 words; words 0 and 32 (128 B apart) are the two mailboxes.
// out[4*wg + k]: k=0 xcc id, 1 iterations completed, 2 elapsed ticks, 3 timed out
__global__ void k_pp(uint32_t* buf, uint32_t* out, int wa, int wb, int iters, int lpol, int spol)
{
    const int wg = blockIdx.x;
    uint32_t xcc;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
    if (threadIdx.x == 0)
        out[4 * wg] = xcc & 0xf;
    if (threadIdx.x != 0 || (wg != wa && wg != wb))
        return;
    __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(buf, (short)0, 256, 0x00020000);
    const bool a = wg == wa;
    const int mine = a ? 0 : 128, theirs = a ? 128 : 0; // byte offsets
    const uint64_t t0 = wclk();
    int done = 0, to = 0;
    for (int n = 1; n <= iters; ++n) {
        // a sends n, then waits for b's n; b waits for a's n, then sends n
        if (a)
            st(r, mine, (uint32_t)n, spol);
        uint32_t polls = 0;
        while (ld(r, theirs, lpol) != (uint32_t)n) {
            if (++polls > 2000000u || wclk() - t0 > 200000000ull) { // 2 s
                to = 1;
                break;
            }
        }
        if (to)
            break;
        if (!a)
            st(r, mine, (uint32_t)n, spol);
        done = n;
    }
    out[4 * wg + 1] = done;
    out[4 * wg + 2] = (uint32_t)(wclk() - t0);
    out[4 * wg + 3] = to;
}

int main()
{
    uint32_t *buf, *out;
    const int G = 64;
    hipMalloc(&buf, 256);
    hipMalloc(&out, 4 * G * 4);
    uint32_t h[4 * G];
    const int pols[][2] = {{16, 16}, {1, 0}, {1, 1}, {17, 17}, {16, 0}, {1, 16}};
    const int iters = 2000;
    for (int pair = 0; pair < 3; ++pair) {
        for (auto& p : pols) {
            const int wa = 0, wb = pair == 0 ? 8 : pair == 1 ? 1 : 4;
            hipMemset(buf, 0, 256);
            hipMemset(out, 0, 4 * G * 4);
            hipDeviceSynchronize();
            hipLaunchKernelGGL(k_pp, dim3(G), dim3(64), 0, 0, buf, out, wa, wb, iters, p[0], p[1]);
            if (hipDeviceSynchronize() != hipSuccess) { printf("launch failed\n"); return 1; }
            hipMemcpy(h, out, sizeof h, hipMemcpyDeviceToHost);
            printf("wg %d (xcc %u) <-> wg %d (xcc %u)  load pol %2d store pol %2d : %u/%d round trips, %s, %.1f ns per round trip\n",
                   wa, h[4 * wa], wb, h[4 * wb], p[0], p[1], h[4 * wa + 1], iters,
                   (h[4 * wa + 3] | h[4 * wb + 3]) ? "TIMED OUT" : "ok",
                   h[4 * wa + 1] ? h[4 * wa + 2] * 10.0 / h[4 * wa + 1] : 0.0);
        }
    }
    printf("xcc of wg 0..15:");
    for (int g = 0; g < 16; ++g) printf(" %u", h[4 * g]);
    printf("\n");
    return 0;
}
