// Measurement probe (not part of the library): LDS throughput of the
// accumulation primitives the forward projector can use, in lanes per clock
// per CU on one GPU: FP32 and FP64 atomic adds (ds_add_f32, ds_add_f64; the
// build must pass -munsafe-fp-atomics so FP32 adds are native instructions,
// not compare-and-swap loops) and plain read-add-write sequences, for a
// wavefront touching 64 distinct addresses one element apart (no bank
// conflicts) and two elements apart (16 bytes: two-way conflicts for FP64).
//
//   hipcc -O3 --offload-arch=gfx950 -munsafe-fp-atomics -o /tmp/lds_atomics \
//       paper_1401_3615_amd/probes/lds_atomics.hip && /tmp/lds_atomics
#include <hip/hip_runtime.h>

#include <cstdio>

template <typename T, bool ATOMIC>
__global__ __launch_bounds__(256) void probe(T* out, int iters, int stride)
{
    __shared__ T buf[8192];
    for (int i = threadIdx.x; i < 8192; i += 256) buf[i] = 0;
    __syncthreads();
    int a = (threadIdx.x * stride) & 4095;
    const T v = (T)1;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            T* p = buf + ((a + u * 97) & 4095);
            if (ATOMIC) __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            else *p += v;
        }
        a = (a + 13) & 4095;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 8192; i += 256) out[(size_t)blockIdx.x * 8192 + i] = buf[i];
}

template <typename T, bool ATOMIC>
static void run(const char* name, int stride, int cus, double ghz)
{
    const int blocks = cus * 16, iters = 2000;
    T* out = nullptr;
    if (hipMalloc(&out, sizeof(T) * 8192 * (size_t)blocks) != hipSuccess) return;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    probe<T, ATOMIC><<<blocks, 256>>>(out, 10, stride);
    (void)hipEventRecord(e0);
    probe<T, ATOMIC><<<blocks, 256>>>(out, iters, stride);
    (void)hipEventRecord(e1);
    (void)hipEventSynchronize(e1);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double ops = (double)blocks * 256 * iters * 8;
    printf("%-22s stride %d: %8.3f ms, %6.2f lanes/clk/CU\n", name, stride, ms, ops / (ms * 1e-3) / (ghz * 1e9) / cus);
    (void)hipFree(out);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

int main()
{
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, 0) != hipSuccess) return 1;
    const double ghz = p.clockRate / 1e6;
    printf("%s, %d CUs, %.2f GHz\n", p.gcnArchName, p.multiProcessorCount, ghz);
    for (int stride : {1, 2}) {
        run<float, true>("ds_add_f32", stride, p.multiProcessorCount, ghz);
        run<double, true>("ds_add_f64", stride, p.multiProcessorCount, ghz);
        run<float, false>("f32 read-add-write", stride, p.multiProcessorCount, ghz);
        run<double, false>("f64 read-add-write", stride, p.multiProcessorCount, ghz);
    }
    return 0;
}
