// Instruction-rate loops behind the sweep's VALU roofline: integer adds (the
// full-rate reference), 32 x 32 -> 64 multiply-adds and whole Philox4x32-10
// calls, each over independent dependency chains per lane so that the issue
// rate, not latency, is measured.  C ABI in include/pdg_rates.h.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pdg.h"
#include "pdg_rates.h"
#include "pdg_rng.hpp"

namespace pdgr {

constexpr int kChains = 16;

__global__ __launch_bounds__(256) void k_rate_add(int64_t iters, uint32_t seed, uint32_t *out)
{
    uint32_t x[kChains], y[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
        x[i] = threadIdx.x * 7u + (uint32_t)i + seed;
        y[i] = blockIdx.x + (uint32_t)i * 3u;
    }
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) {
            x[i] += y[i];  // one v_add_u32 each: kChains / 2 pairs of chains
            y[i] += x[i];
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) acc ^= x[i] ^ y[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_rate_mad64(int64_t iters, uint32_t seed, uint32_t *out)
{
    uint64_t p[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) p[i] = (uint64_t)(threadIdx.x * 13u + (uint32_t)i + seed);
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i)
            p[i] = (uint64_t)0xD2511F53u * (uint64_t)(uint32_t)p[i] + (p[i] >> 32);
    }
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) acc ^= (uint32_t)p[i] ^ (uint32_t)(p[i] >> 32);
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_rate_philox(int64_t iters, uint32_t seed, uint32_t *out,
                                                      pdg::RoundKeys rk)
{
    constexpr int NS = 4;  // independent streams per lane
    uint32_t c[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) c[i] = threadIdx.x + (uint32_t)i * 977u + seed;
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            const pdg::Words w = pdg::philox4x32_10(c[i], blockIdx.x, (uint32_t)it, (uint32_t)i, rk);
            c[i] = w.w0 ^ w.w3;
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < NS; ++i) acc ^= c[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

}  // namespace pdgr

extern "C" pdg_status pdg_valu_rates(int32_t device, int64_t iters, double *h_out)
{
    if (!h_out || iters < 1 || iters > (1 << 24)) return PDG_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return PDG_EHIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return PDG_EHIP;
    // eight waves per SIMD on every compute unit
    const unsigned blocks = (unsigned)prop.multiProcessorCount * 8u;
    const unsigned threads = 256u;
    const double lanes = (double)blocks * threads;
    uint32_t *d_out = nullptr;
    if (hipMalloc(&d_out, (size_t)blocks * threads * 4) != hipSuccess) return PDG_EHIP;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        (void)hipFree(d_out);
        return PDG_EHIP;
    }
    const pdg::RoundKeys rk = pdg::make_round_keys(0x243F6A8885A308D3ull);
    auto timed = [&](int which, int64_t n) -> double {
        for (int rep = 0; rep < 2; ++rep) {  // warm-up, then the timed launch
            (void)hipEventRecord(a, 0);
            if (which == 0)
                pdgr::k_rate_add<<<blocks, threads>>>(n, 1u, d_out);
            else if (which == 1)
                pdgr::k_rate_mad64<<<blocks, threads>>>(n, 2u, d_out);
            else
                pdgr::k_rate_philox<<<blocks, threads>>>(n, 3u, d_out, rk);
            (void)hipEventRecord(b, 0);
        }
        (void)hipEventSynchronize(b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        return (double)ms;
    };
    const double ms_add = timed(0, iters), ms_mad = timed(1, iters), ms_phx = timed(2, iters / 16 + 1);
    const hipError_t e = hipGetLastError();
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(d_out);
    if (e != hipSuccess) return PDG_EHIP;
    h_out[0] = lanes * (double)iters * 2.0 * pdgr::kChains / (ms_add * 1e-3);
    h_out[1] = lanes * (double)iters * pdgr::kChains / (ms_mad * 1e-3);
    h_out[2] = lanes * (double)(iters / 16 + 1) * 4.0 / (ms_phx * 1e-3);
    return PDG_OK;
}
