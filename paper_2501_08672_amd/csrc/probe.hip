// Measurement aid for the roofline of the compositing kernels (not a step of
// the method): how many wave64 VALU instructions per CU and cycle the chip
// issues for a given instruction kind, with every SIMD holding eight waves of
// eight independent dependency chains.  The compositing walks are bound by
// VALU issue, and their mix of fused multiply-adds, transcendentals and
// single-cycle integer / select / add instructions meets these ceilings.
#include "common.hpp"

namespace gsl {

namespace {

constexpr int kProbeChains = 8;

// mode 0: one FP32 fused multiply-add per chain and iteration;
// mode 1: an FP32 multiply and a v_exp_f32 per chain and iteration;
// mode 2: an unsigned min and an FP32 add per chain and iteration;
// mode 3: one FP32 add per chain and iteration;
// mode 4: one FP32 multiply per chain and iteration.
// The result is stored only if negative, which no chain becomes, so the
// loop cannot be removed and nothing is written.
template <int MODE>
__global__ __launch_bounds__(256) void k_valu_probe(float *__restrict__ sink, int iters, float b, float c)
{
    float x[kProbeChains];
#pragma unroll
    for (int i = 0; i < kProbeChains; i++) x[i] = 1.0f + 1e-3f * (float)(threadIdx.x & 15) + 0.125f * (float)i;
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int i = 0; i < kProbeChains; i++) {
            if (MODE == 0) x[i] = fmaf(x[i], b, c);
            if (MODE == 1) x[i] = __builtin_amdgcn_exp2f(x[i] * b);
            if (MODE == 2) x[i] = __uint_as_float(min(__float_as_uint(x[i]), 0x3f800000u)) + c;
            if (MODE == 3) x[i] = x[i] + c;
            if (MODE == 4) x[i] = x[i] * b;
        }
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < kProbeChains; i++) s += x[i];
    if (s < 0.f) sink[0] = s;
}

}  // namespace

int run_valu_probe(int mode, int num_cus, float *sink, double *rate)
{
    constexpr int kIters = 4096, kReps = 5;
    const int blocks = num_cus * 8;  // eight 4-wave workgroups per CU: eight waves per SIMD
    auto launch = [&](hipStream_t s) {
        // b and c keep every chain positive and finite (x -> c / (1 - b), exp2 of a value below 1, min then
        // add, a slow climb by c, a slow decay by b)
        if (mode == 0) hipLaunchKernelGGL(k_valu_probe<0>, dim3(blocks), dim3(256), 0, s, sink, kIters, 0.999f, 1e-4f);
        if (mode == 1) hipLaunchKernelGGL(k_valu_probe<1>, dim3(blocks), dim3(256), 0, s, sink, kIters, 0.5f, 1e-4f);
        if (mode == 2) hipLaunchKernelGGL(k_valu_probe<2>, dim3(blocks), dim3(256), 0, s, sink, kIters, 0.999f, 1e-4f);
        if (mode == 3) hipLaunchKernelGGL(k_valu_probe<3>, dim3(blocks), dim3(256), 0, s, sink, kIters, 0.999f, 1e-4f);
        if (mode == 4) hipLaunchKernelGGL(k_valu_probe<4>, dim3(blocks), dim3(256), 0, s, sink, kIters, 0.999f, 1e-4f);
    };
    hipStream_t s = nullptr;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1;
    }
    launch(s);  // warm-up
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < kReps; r++) launch(s);
    (void)hipEventRecord(e1, s);
    float ms = 0.f;
    hipError_t err = hipEventSynchronize(e1);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess || ms <= 0.f) return -1;
    // wave64 VALU instructions of the loop: 16 per iteration in modes 1 and 2, 8 in the others
    const double per_wave = (mode == 1 || mode == 2 ? 16.0 : 8.0) * kIters;
    const double insts = per_wave * blocks * 4.0 * kReps;
    const double cu_cycles = (double)num_cus * (ms * 1e-3) * 2.4e9;
    *rate = insts / cu_cycles;
    return 0;
}

}  // namespace gsl
