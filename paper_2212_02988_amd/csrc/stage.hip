// Frame staging for serving: one kernel copies a frame (depth, rgb, control)
// from wherever the caller keeps it on the device into a stream's fixed input
// slot, so the slot's recorded step graph can be replayed.
#include "common.hpp"
#include "launch.hpp"

namespace prism {

// vec: all pointers 16-byte aligned and npix a multiple of 4 (float4 copies)
__global__ __launch_bounds__(256) void k_stage(const float* __restrict__ d_in, const float* __restrict__ c_in,
                                               const double* __restrict__ u_in, float* __restrict__ d_out,
                                               float* __restrict__ c_out, double* __restrict__ u_out,
                                               long long npix, int vec) {
    long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    if (u_in && tid < 6) u_out[tid] = u_in[tid];
    if (vec) {
        long long nd = npix >> 2, nc = (3 * npix) >> 2;
        const float4* d4 = reinterpret_cast<const float4*>(d_in);
        const float4* c4 = reinterpret_cast<const float4*>(c_in);
        float4* do4 = reinterpret_cast<float4*>(d_out);
        float4* co4 = reinterpret_cast<float4*>(c_out);
        for (long long i = tid; i < nc; i += stride) {
            co4[i] = c4[i];
            if (i < nd) do4[i] = d4[i];
        }
    } else {
        for (long long i = tid; i < 3 * npix; i += stride) {
            c_out[i] = c_in[i];
            if (i < npix) d_out[i] = d_in[i];
        }
    }
}

// batched: filter a's frame into its slot, workgroups [start[a], start[a+1])
// striding over the frame (vectorised when every pointer allows it)
__global__ __launch_bounds__(256) void k_stage_batch(BatchArgs b, StageSrc src) {
    const int a = batch_agent(b, blockIdx.x);
    const AgentDesc& D = *b.d[a];
    const prism_frame& slot = D.slots[b.slot[a]];
    const long long npix = (long long)D.c.W * D.c.H;
    const int nblk = b.start[a + 1] - b.start[a];
    const long long tid = (long long)(blockIdx.x - b.start[a]) * blockDim.x + threadIdx.x;
    const long long stride = (long long)nblk * blockDim.x;
    const float* d_in = (const float*)src.depth[a];
    const float* c_in = (const float*)src.rgb[a];
    const double* u_in = (const double*)src.u[a];
    float* d_out = (float*)slot.depth;
    float* c_out = (float*)slot.rgb;
    if (u_in && tid < 6) ((double*)slot.u)[tid] = u_in[tid];
    auto a16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    if ((npix & 3) == 0 && a16(d_in) && a16(c_in) && a16(d_out) && a16(c_out)) {
        long long nd = npix >> 2, nc = (3 * npix) >> 2;
        const float4* d4 = reinterpret_cast<const float4*>(d_in);
        const float4* c4 = reinterpret_cast<const float4*>(c_in);
        float4* do4 = reinterpret_cast<float4*>(d_out);
        float4* co4 = reinterpret_cast<float4*>(c_out);
        for (long long i = tid; i < nc; i += stride) {
            co4[i] = c4[i];
            if (i < nd) do4[i] = d4[i];
        }
    } else {
        for (long long i = tid; i < 3 * npix; i += stride) {
            c_out[i] = c_in[i];
            if (i < npix) d_out[i] = d_in[i];
        }
    }
}

// workgroups per filter of the batched staging kernel
int stage_blocks(const CamC& c) {
    long long work = (3LL * c.W * c.H) / 4;
    long long blocks = (work + 255) / 256;
    return (int)(blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks));
}

hipError_t launch_stage_batch(const BatchArgs& b, const StageSrc& src, hipStream_t st) {
    k_stage_batch<<<b.start[b.n], 256, 0, st>>>(b, src);
    return hipGetLastError();
}

hipError_t launch_stage(const void* depth, const void* rgb, const void* u, float* d_out, float* c_out, double* u_out,
                        long long npix, hipStream_t st) {
    auto a16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    int vec = (npix % 4 == 0) && a16(depth) && a16(rgb) && a16(d_out) && a16(c_out);
    long long work = vec ? (3 * npix) / 4 : 3 * npix;
    long long blocks = (work + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    k_stage<<<(unsigned)blocks, 256, 0, st>>>((const float*)depth, (const float*)rgb, (const double*)u, d_out, c_out,
                                             u_out, npix, vec);
    return hipGetLastError();
}

}  // namespace prism
