// LDS throughput of the ring kernel's access: 16-byte elements (an FP64
// complex value) read with ds_read_b128 and written with ds_write_b128, at
// the padded slots i + i/8 of a 4096-element buffer, eight accesses per lane
// 512 elements apart (the pattern of a radix-8 pass).  Two workgroups of 512
// threads per CU, as in the ring kernel's smaller-buffer launch.  Prints the
// chip-wide rates that bench.py takes as the LDS roofline of the ring step.
//
// build and run:  hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops
//                    -o lds_probe bench_lds_probe.hip && ./lds_probe
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                    \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) {                                                     \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));            \
            std::exit(1);                                                           \
        }                                                                           \
    } while (0)

constexpr int kElems = 4096;
constexpr int kSlots = kElems + kElems / 8;

// WRITE = false: each lane reads its eight elements and sums them;
// WRITE = true: each lane writes eight elements.  Addresses depend on the
// lane and the iteration only, and stay below kSlots.
template <bool WRITE>
__global__ __launch_bounds__(512) void lds_kernel(double* out, int iters) {
    __shared__ double2 buf[kSlots];
    const int t = threadIdx.x;
    for (int i = t; i < kSlots; i += blockDim.x) buf[i] = make_double2(i, -i);
    __syncthreads();
    double2 acc = make_double2(0, 0);
    int idx = t;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int k = (idx + c * 512) & (kElems - 1);
            const int p = k + (k >> 3);
            if (!WRITE) {
                const double2 v = buf[p];
                acc.x += v.x;
                acc.y += v.y;
            } else {
                buf[p] = make_double2(acc.x + c, acc.y - c);
            }
        }
        idx = (idx + 37) & (kElems - 1);
        if (WRITE) acc.x += 1.0;
    }
    if (WRITE) {
        __syncthreads();
        acc = buf[t];
    }
    out[blockIdx.x * blockDim.x + t] = acc.x + acc.y;
}

int main() {
    int dev = 0, cus = 0;
    CHECK(hipGetDevice(&dev));
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int threads = 512, blocks = 2 * cus, iters = 4000;
    double* d = nullptr;
    CHECK(hipMalloc(&d, sizeof(double) * blocks * threads));
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    const double bytes = (double)blocks * threads * iters * 8 * 16;
    for (int write = 0; write < 2; ++write) {
        float best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            CHECK(hipEventRecord(a));
            if (write) hipLaunchKernelGGL(lds_kernel<true>, dim3(blocks), dim3(threads), 0, 0, d, iters);
            else hipLaunchKernelGGL(lds_kernel<false>, dim3(blocks), dim3(threads), 0, 0, d, iters);
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(b));
            CHECK(hipEventSynchronize(b));
            float ms = 0;
            CHECK(hipEventElapsedTime(&ms, a, b));
            if (ms < best) best = ms;
        }
        std::printf("%s_TBps: %.2f\n", write ? "write" : "read", bytes / best / 1e9);
        std::printf("%s_bytes_per_clk_per_cu_at_2p4GHz: %.1f\n", write ? "write" : "read",
                    bytes / (best * 1e-3) / cus / 2.4e9);
    }
    std::vector<double> h(blocks * threads);
    CHECK(hipMemcpy(h.data(), d, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
    std::printf("cus: %d\nchecksum: %g\n", cus, h[0] + h[h.size() - 1]);
    CHECK(hipFree(d));
    return 0;
}
