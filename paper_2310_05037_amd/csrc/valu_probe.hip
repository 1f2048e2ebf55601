// valu_probe.hip -- issue-rate probe behind the roofline peak of the DTW
// kernels (libvaluprobe.so, loaded by bench.py --valu-rate; not part of the
// alignment library).
//
// Every wave runs eight independent chains of one VALU instruction form for
// `iters` rounds and reads the shader-clock counter before and after, so the
// rate comes out in lane-operations per clock per CU without knowing the
// clock.  The forms are written as inline assembly (VALU only, no memory
// access inside the timed loop), so the compiler can neither merge nor
// reassociate them:
//   0  v_add_f32             (pairs with another VALU op in dual issue)
//   1  v_sub_f32
//   2  v_min3_f32
//   3  v_max_f32
//   4  the DTW cell: v_sub_f32, v_min3_f32, v_add_f32 with an |x| source
//      modifier (three instructions, three lane-operations per cell)
#include <hip/hip_runtime.h>

#include <chrono>
#include <thread>
#include <stdint.h>

namespace {

constexpr int kChains = 8;

template <int OP>
__device__ __forceinline__ void round8(float (&a)[kChains], const float (&x)[kChains], const float (&y)[kChains]) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
        if constexpr (OP == 0) {
            asm volatile("v_add_f32 %0, %0, %1" : "+v"(a[k]) : "v"(x[k]));
        } else if constexpr (OP == 1) {
            asm volatile("v_sub_f32 %0, %0, %1" : "+v"(a[k]) : "v"(x[k]));
        } else if constexpr (OP == 2) {
            asm volatile("v_min3_f32 %0, %0, %1, %2" : "+v"(a[k]) : "v"(x[k]), "v"(y[k]));
        } else if constexpr (OP == 3) {
            asm volatile("v_max_f32 %0, %0, %1" : "+v"(a[k]) : "v"(x[k]));
        } else {
            float d;
            asm volatile("v_sub_f32 %0, %1, %2" : "=v"(d) : "v"(x[k]), "v"(y[k]));
            asm volatile("v_min3_f32 %0, %0, %1, %2" : "+v"(a[k]) : "v"(x[k]), "v"(y[k]));
            asm volatile("v_add_f32 %0, |%1|, %0" : "+v"(a[k]) : "v"(d));
        }
    }
}

template <int OP>
__global__ __launch_bounds__(64) void k_probe(int iters, float seed, float *sink, uint64_t *cycles) {
    float a[kChains], x[kChains], y[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
        a[k] = seed * (float)(threadIdx.x + k);
        x[k] = seed + (float)k;
        y[k] = seed - (float)k;
    }
    __builtin_amdgcn_s_waitcnt(0);
    const uint64_t t0 = clock64();
    for (int it = 0; it < iters; ++it) round8<OP>(a, x, y);
    const uint64_t t1 = clock64();
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += a[k];
    sink[blockIdx.x * 64 + threadIdx.x] = s;
    if (threadIdx.x == 0) cycles[blockIdx.x] = t1 - t0;
}

template <int OP>
hipError_t launch(int blocks, int iters, float *sink, uint64_t *cycles) {
    hipLaunchKernelGGL(k_probe<OP>, dim3(blocks), dim3(64), 0, 0, iters, 1.0f / 1024.0f, sink, cycles);
    return hipGetLastError();
}

// One thread reads the constant-rate clock that the pipelined kernels'
// capped waits measure time with, and the shader cycle counter.
__global__ void k_clock(uint64_t *out) {
    if (threadIdx.x == 0) {
        out[0] = __builtin_amdgcn_s_memrealtime();
        out[1] = __builtin_amdgcn_s_memtime();
    }
}

}  // namespace

extern "C" {

// Rate of s_memrealtime: two one-thread launches `sleep_ms` of host wall
// time apart; *ticks receives the clock difference, *seconds the host time
// between the two reads' completions.  Returns 0, -1 for a bad argument, -2
// for a HIP error.
int clock_probe(int sleep_ms, double *ticks, double *seconds) {
    if (sleep_ms < 1 || sleep_ms > 10000) return -1;
    uint64_t *d = nullptr;
    if (hipMalloc(&d, 4 * sizeof(uint64_t)) != hipSuccess) return -2;
    uint64_t h[4] = {0, 0, 0, 0};
    hipError_t e = hipSuccess;
    std::chrono::steady_clock::time_point t0, t1;
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        hipLaunchKernelGGL(k_clock, dim3(1), dim3(64), 0, 0, d + 2 * k);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (k == 0) {
            t0 = std::chrono::steady_clock::now();
            std::this_thread::sleep_for(std::chrono::milliseconds(sleep_ms));
        } else {
            t1 = std::chrono::steady_clock::now();
        }
    }
    if (e == hipSuccess) e = hipMemcpy(h, d, sizeof(h), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return -2;
    *ticks = (double)(h[2] - h[0]);
    *seconds = std::chrono::duration<double>(t1 - t0).count();
    return 0;
}

// Lane-operations per clock per CU of form `op` (see above) with
// `waves_per_cu` single-wave workgroups on every CU, and the shader clock
// implied by the counter (cycles of the slowest wave / kernel time).
// Returns 0, or -1 for a bad argument, -2 for a HIP error.
int valu_probe(int op, int waves_per_cu, int iters, double *lane_ops_per_clk_per_cu, double *clock_ghz,
               double *kernel_ms) {
    if (op < 0 || op > 4 || waves_per_cu < 1 || waves_per_cu > 32 || iters < 1) return -1;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return -2;
    const int cus = prop.multiProcessorCount;
    const int blocks = cus * waves_per_cu;
    float *sink = nullptr;
    uint64_t *cycles = nullptr;
    if (hipMalloc(&sink, sizeof(float) * 64 * (size_t)blocks) != hipSuccess) return -2;
    if (hipMalloc(&cycles, sizeof(uint64_t) * (size_t)blocks) != hipSuccess) {
        (void)hipFree(sink);
        return -2;
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    hipError_t (*fn)(int, int, float *, uint64_t *) =
        op == 0 ? launch<0> : op == 1 ? launch<1> : op == 2 ? launch<2> : op == 3 ? launch<3> : launch<4>;
    hipError_t e = fn(blocks, iters, sink, cycles);   // warm-up
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipEventRecord(e0, 0);
    if (e == hipSuccess) e = fn(blocks, iters, sink, cycles);
    if (e == hipSuccess) e = hipEventRecord(e1, 0);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    uint64_t *h = new uint64_t[blocks];
    if (e == hipSuccess) e = hipMemcpy(h, cycles, sizeof(uint64_t) * (size_t)blocks, hipMemcpyDeviceToHost);
    if (e == hipSuccess) {
        uint64_t mx = 0;
        for (int i = 0; i < blocks; ++i) mx = h[i] > mx ? h[i] : mx;
        const double ops_per_round = op == 4 ? 3.0 : 1.0;
        const double lane_ops_wave = 64.0 * kChains * ops_per_round * (double)iters;
        *lane_ops_per_clk_per_cu = lane_ops_wave * waves_per_cu / (double)mx;
        *clock_ghz = (double)mx / (ms * 1e6);
        *kernel_ms = ms;
    }
    delete[] h;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    (void)hipFree(cycles);
    return e == hipSuccess ? 0 : -2;
}

}  // extern "C"
