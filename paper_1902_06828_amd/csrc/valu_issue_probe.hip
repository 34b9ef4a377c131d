// VALU issue rates of the instruction forms the KSG kernels use (gfx950).
//
//     paper_1902_06828_amd/valu_issue_probe      (built by build.py)
//
// Each lane runs 8 independent chains of one instruction form (or of one
// short sequence) for kIter trips, on grids of 1, 2, 4 and 8 waves per SIMD;
// the shortest of five launches gives lane-instructions per second.  It backs
// the ALU peaks the benchmark prices its kernels against: float add, subtract
// and fma and the simple integer forms issue at 128 lanes per clock per CU,
// while min, max, med3, the three-operand forms and compares issue at 64.
// Every thread writes one float (index < grid x 256, the buffer holds the
// largest grid); the loops have fixed trip counts.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <vector>

#define CHK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { printf("HIP error %s at %d\n", hipGetErrorString(e_), __LINE__); return 1; } } while (0)

constexpr int kIter = 4096;   // loop trips; 8 chains x UNR instructions each

template <int OP>
__global__ __launch_bounds__(256) void probe(float *out, float b, float c) {
    float a[8];
    int ci[8];
    int ti[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) { a[k] = threadIdx.x * 0.001f + k; ci[k] = 0; ti[k] = 0; }
    for (int it = 0; it < kIter; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if constexpr (OP == 0) asm volatile("v_max_f32 %0, %0, |%1|" : "+v"(a[k]) : "v"(b));
            if constexpr (OP == 1) asm volatile("v_sub_f32 %0, %0, %1" : "+v"(a[k]) : "v"(b));
            if constexpr (OP == 2) asm volatile("v_cmp_lt_f32_e32 vcc, %1, %2\n\tv_addc_co_u32_e32 %0, vcc, 0, %0, vcc" : "+v"(ci[k]) : "v"(a[k]), "v"(b) : "vcc");
            if constexpr (OP == 3) asm volatile("v_med3_f32 %0, %0, %1, %2" : "+v"(a[k]) : "v"(b), "v"(c));
            if constexpr (OP == 4) asm volatile("v_max3_f32 %0, %0, |%1|, |%2|" : "+v"(a[k]) : "v"(b), "v"(c));
            if constexpr (OP == 5) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a[k]) : "v"(b), "v"(c));
            if constexpr (OP == 6) asm volatile("v_add_f32 %0, %0, %1" : "+v"(a[k]) : "v"(b));
            if constexpr (OP == 7) asm volatile("v_min_f32 %0, %0, %1" : "+v"(a[k]) : "v"(b));
            if constexpr (OP == 8) asm volatile("v_cmp_lt_f32_e32 vcc, %1, %2\n\tv_cndmask_b32_e32 %0, %0, %1, vcc" : "+v"(a[k]) : "v"(b), "v"(c) : "vcc");
            if constexpr (OP == 9) asm volatile("v_sub_u32 %0, %0, %1" : "+v"(ci[k]) : "v"(b));
            if constexpr (OP == 10) asm volatile("v_lshrrev_b32 %0, 31, %0" : "+v"(ci[k]));
            if constexpr (OP == 11) asm volatile("v_add_u32 %0, %0, %1" : "+v"(ci[k]) : "v"(b));
            if constexpr (OP == 12) asm volatile("v_and_b32 %0, %0, %1" : "+v"(ci[k]) : "v"(b));
            if constexpr (OP == 13) asm volatile("v_max_u32 %0, %0, %1" : "+v"(ci[k]) : "v"(b));
            if constexpr (OP == 14) asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(ci[k]) : "v"(b), "v"(c));
            if constexpr (OP == 15) asm volatile("v_max3_u32 %0, %0, %1, %2" : "+v"(ci[k]) : "v"(b), "v"(c));
            if constexpr (OP == 16) asm volatile("v_sub_u32 %0, %2, %3\n\tv_lshrrev_b32 %0, 31, %0\n\tv_add_u32 %1, %1, %0" : "=&v"(ti[k]), "+v"(ci[k]) : "v"(a[k]), "v"(c));
            if constexpr (OP == 17) asm volatile("v_lshl_add_u32 %0, %0, 1, %1" : "+v"(ci[k]) : "v"(b));
            if constexpr (OP == 18) asm volatile("v_bfe_u32 %0, %0, 31, 1" : "+v"(ci[k]));
        }
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += a[k] + (float)ci[k] + (float)ti[k];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <int OP>
static int run(const char *name, int instr_per_chain_step, float *d_out, int n_cu) {
    hipEvent_t e0, e1;
    CHK(hipEventCreate(&e0));
    CHK(hipEventCreate(&e1));
    for (int wps = 1; wps <= 8; wps *= 2) {
        const int blocks = n_cu * wps;           // 4 waves per block -> wps waves per SIMD
        hipLaunchKernelGGL(probe<OP>, dim3(blocks), dim3(256), 0, 0, d_out, 1.5f, 0.25f);
        CHK(hipGetLastError());
        CHK(hipDeviceSynchronize());
        float best = 1e30f;
        for (int r = 0; r < 5; ++r) {
            CHK(hipEventRecord(e0, 0));
            hipLaunchKernelGGL(probe<OP>, dim3(blocks), dim3(256), 0, 0, d_out, 1.5f, 0.25f);
            CHK(hipEventRecord(e1, 0));
            CHK(hipEventSynchronize(e1));
            float ms = 0.f;
            CHK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) best = ms;
        }
        const double lane_instr = (double)blocks * 256.0 * kIter * 8.0 * instr_per_chain_step;
        printf("%-22s waves/SIMD %d: %.4f ms, %.1f T lane-instr/s\n", name, wps, best, lane_instr / (best * 1e-3) / 1e12);
        fflush(stdout);
    }
    CHK(hipEventDestroy(e0));
    CHK(hipEventDestroy(e1));
    return 0;
}

int main() {
    int n_cu = 0;
    CHK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, 0));
    hipDeviceProp_t p;
    CHK(hipGetDeviceProperties(&p, 0));
    printf("device %s, %d CUs, clock %d kHz\n", p.gcnArchName, n_cu, p.clockRate);
    float *d_out = nullptr;
    CHK(hipMalloc(&d_out, sizeof(float) * (size_t)n_cu * 8 * 256));
    int rc = 0;
    rc |= run<0>("v_max_f32 abs(b)", 1, d_out, n_cu);
    rc |= run<1>("v_sub_f32", 1, d_out, n_cu);
    rc |= run<2>("v_cmp_lt + v_addc", 2, d_out, n_cu);
    rc |= run<3>("v_med3_f32", 1, d_out, n_cu);
    rc |= run<4>("v_max3_f32 abs(b) abs(c)", 1, d_out, n_cu);
    rc |= run<5>("v_fma_f32", 1, d_out, n_cu);
    rc |= run<6>("v_add_f32", 1, d_out, n_cu);
    rc |= run<7>("v_min_f32", 1, d_out, n_cu);
    rc |= run<8>("v_cmp_lt + v_cndmask", 2, d_out, n_cu);
    rc |= run<9>("v_sub_u32", 1, d_out, n_cu);
    rc |= run<10>("v_lshrrev_b32", 1, d_out, n_cu);
    rc |= run<11>("v_add_u32", 1, d_out, n_cu);
    rc |= run<12>("v_and_b32", 1, d_out, n_cu);
    rc |= run<13>("v_max_u32", 1, d_out, n_cu);
    rc |= run<14>("v_add3_u32", 1, d_out, n_cu);
    rc |= run<15>("v_max3_u32", 1, d_out, n_cu);
    rc |= run<16>("sub + lshr + add (count)", 3, d_out, n_cu);
    rc |= run<17>("v_lshl_add_u32", 1, d_out, n_cu);
    rc |= run<18>("v_bfe_u32", 1, d_out, n_cu);
    CHK(hipFree(d_out));
    return rc;
}
