// Issue rates of the instructions the 64-bit modular arithmetic is built
// from, on the current GPU: v_mad_u64_u32 (32x32+64), v_mul_lo_u32,
// v_mul_hi_u32, v_add_u32, a whole 64-bit Shoup modular multiplication, the
// binary64 FMA, and a modular multiplication in binary64 arithmetic for
// primes below 2^41 (product split exactly by an FMA, quotient rounded from
// a precomputed w/q, remainder by a second FMA).  Each thread runs 8
// independent dependency chains so the ALU, not latency, limits the rate.
// Prints one JSON line.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#define CHAINS 8
#define ITERS 4096

// acc <- lo(acc) * hi(acc) + acc: one v_mad_u64_u32 per step (data dependent, not foldable)
__global__ void k_mad64(uint64_t* out, uint32_t a, uint32_t b)
{
    uint64_t acc[CHAINS];
    for (int c = 0; c < CHAINS; ++c) acc[c] = ((uint64_t)(a + threadIdx.x + c) << 32) | (b + c);
    for (int i = 0; i < ITERS; ++i)
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) acc[c] = (uint64_t)(uint32_t)acc[c] * (uint32_t)(acc[c] >> 32) + acc[c];
    uint64_t s = 0;
    for (int c = 0; c < CHAINS; ++c) s ^= acc[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void k_mullo(uint64_t* out, uint32_t a, uint32_t b)
{
    uint32_t acc[CHAINS];
    for (int c = 0; c < CHAINS; ++c) acc[c] = a + threadIdx.x + c;
    for (int i = 0; i < ITERS; ++i)
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) acc[c] = acc[c] * (acc[c] ^ b);  // v_mul_lo_u32 + v_xor
    uint32_t s = 0;
    for (int c = 0; c < CHAINS; ++c) s ^= acc[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void k_mulhi(uint64_t* out, uint32_t a, uint32_t b)
{
    uint32_t acc[CHAINS];
    for (int c = 0; c < CHAINS; ++c) acc[c] = a + threadIdx.x + c;
    for (int i = 0; i < ITERS; ++i)
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) acc[c] = __umulhi(acc[c], acc[c] ^ b);  // v_mul_hi_u32 + v_xor
    uint32_t s = 0;
    for (int c = 0; c < CHAINS; ++c) s ^= acc[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void k_add(uint64_t* out, uint32_t a, uint32_t b)
{
    uint32_t acc[CHAINS];
    for (int c = 0; c < CHAINS; ++c) acc[c] = a + threadIdx.x + c;
    for (int i = 0; i < ITERS; ++i)
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) acc[c] = (acc[c] + b) ^ (acc[c] >> 7);  // add, shift, xor
    uint32_t s = 0;
    for (int c = 0; c < CHAINS; ++c) s ^= acc[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// x <- x * w mod q (Shoup, q < 2^61), lazily reduced in [0, 2q)
__global__ void k_shoup(uint64_t* out, uint64_t q, uint64_t w, uint64_t wsh)
{
    uint64_t acc[CHAINS];
    for (int c = 0; c < CHAINS; ++c) acc[c] = (threadIdx.x * 7919u + c) % q;
    for (int i = 0; i < ITERS; ++i)
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) {
            uint64_t qh = __umul64hi(acc[c], wsh);
            acc[c] = acc[c] * w - qh * q;
            acc[c] = acc[c] >= q ? acc[c] - q : acc[c];
        }
    uint64_t s = 0;
    for (int c = 0; c < CHAINS; ++c) s ^= acc[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void k_fma64(uint64_t* out, double a, double b)
{
    double acc[CHAINS];
    for (int c = 0; c < CHAINS; ++c) acc[c] = threadIdx.x + c;
    for (int i = 0; i < ITERS; ++i)
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) acc[c] = __builtin_fma(acc[c], a, b);  // v_fma_f64
    double s = 0;
    for (int c = 0; c < CHAINS; ++c) s += acc[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = (uint64_t)(s != 0.0);
}

// x <- x * w mod q in binary64 (q < 2^41): x stays an integer-valued double
// in (-0.52 q, 0.52 q)
__global__ void k_fpmod(uint64_t* out, double q, double w, double wq)
{
    double acc[CHAINS];
    for (int c = 0; c < CHAINS; ++c) acc[c] = (double)((threadIdx.x * 7919u + c) % 1000003u);
    for (int i = 0; i < ITERS; ++i)
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) {
            const double hi = acc[c] * w;
            const double lo = __builtin_fma(acc[c], w, -hi);
            const double qf = __builtin_rint(acc[c] * wq);
            acc[c] = __builtin_fma(-qf, q, hi) + lo;
        }
    int64_t s = 0;
    for (int c = 0; c < CHAINS; ++c) s ^= (int64_t)acc[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = (uint64_t)s;
}

int main()
{
    hipDeviceProp_t p;
    hipGetDeviceProperties(&p, 0);
    const int blocks = p.multiProcessorCount * 8, threads = 256;
    uint64_t* out;
    if (hipMalloc(&out, sizeof(uint64_t) * blocks * threads) != hipSuccess) return 1;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    const double ops = (double)blocks * threads * ITERS * CHAINS;
    const uint64_t q = 1099510054913ull, w = 123456789012ull;
    const uint64_t wsh = (uint64_t)(((unsigned __int128)w << 64) / q);
    const double qd = (double)q, wd = (double)w;
    double rate[7];
    for (int kind = 0; kind < 7; ++kind) {
        for (int rep = 0; rep < 2; ++rep) {  // first launch warms up
            hipEventRecord(e0, 0);
            switch (kind) {
            case 0: k_mad64<<<blocks, threads>>>(out, 3, 2654435761u); break;
            case 1: k_mullo<<<blocks, threads>>>(out, 3, 2654435761u); break;
            case 2: k_mulhi<<<blocks, threads>>>(out, 3, 2654435761u); break;
            case 3: k_add<<<blocks, threads>>>(out, 3, 2654435761u); break;
            case 4: k_shoup<<<blocks, threads>>>(out, q, w, wsh); break;
            case 5: k_fma64<<<blocks, threads>>>(out, 0.999999, 1e-7); break;
            case 6: k_fpmod<<<blocks, threads>>>(out, qd, wd, wd / qd); break;
            }
            hipEventRecord(e1, 0);
            hipEventSynchronize(e1);
        }
        float ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        rate[kind] = ops / (ms * 1e-3);
    }
    printf("{\"device\": \"%s\", \"cus\": %d, \"clock_mhz\": %d, "
           "\"v_mad_u64_u32_per_s\": %.4e, \"v_mul_lo_u32_per_s\": %.4e, \"v_mul_hi_u32_per_s\": %.4e, "
           "\"v_add_u32_per_s\": %.4e, \"shoup_modmul64_per_s\": %.4e, \"v_fma_f64_per_s\": %.4e, "
           "\"fp64_modmul_per_s\": %.4e}\n",
           p.name, p.multiProcessorCount, p.clockRate / 1000, rate[0], rate[1], rate[2], rate[3], rate[4], rate[5],
           rate[6]);
    hipFree(out);
    return 0;
}
