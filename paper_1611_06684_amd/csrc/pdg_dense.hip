// The dense gather as a matrix product (an experiment on the complete binary
// graphs of the batched workload).  In a binary context with up to 16 chains,
// node i's field of state 1 for chain c is base_i + sum_r 2 theta_r^c h_r over
// its incidence records r: per node a (chains x records) 0/1 matrix times a
// vector, with no operand shared between nodes (each node has its own records
// and duals).  The matrix-core form runs v_mfma_f64_16x16x4_f64 with A = the
// duals of 16 chain rows x 4 records (as 0.0 / 1.0) and B = 2 h of those 4
// records in column 0 of 16 (the other columns zero), so at most 1/16 of each
// product is useful; the vector form is the hub kernels' arithmetic (eight
// record groups of eight chain lanes, one FMA per record and chain, a
// butterfly over the groups).  Both are FP64 and read the same records.
// C ABI in include/pdg_block.h (pdg_dense_fields).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "pdg.h"
#include "pdg_block.h"
#include "pdg_view.hpp"

namespace pdgd {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// one wave per listed node, lane l: chain l % 16 of A's row, record k = l / 16
// of each group of four
__global__ __launch_bounds__(256) void k_dense_mfma(int64_t nn, const int32_t *__restrict__ nodes, int C,
                                                    const double *__restrict__ rec_p,
                                                    const uint32_t *__restrict__ rec_z,
                                                    const uint32_t *__restrict__ off,
                                                    const uint32_t *__restrict__ cnt,
                                                    const double *__restrict__ base,
                                                    double *__restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= nn) return;
    const int64_t i = nodes[w];
    const uint64_t r0 = off[i];
    const uint32_t R = cnt[i];
    const int m = lane & 15, k = lane >> 4;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t k0 = 0; k0 < R; k0 += 4) {
        const uint32_t r = k0 + (uint32_t)k;
        double a = 0.0, b = 0.0;
        if (r < R) {
            const uint32_t z = rec_z[r0 + r];
            a = (m < C && ((z >> m) & 1u)) ? 1.0 : 0.0;
            b = m == 0 ? 2.0 * rec_p[r0 + r] : 0.0;  // B[k][n = lane % 16]
        }
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    // element j of the accumulator is D[row = lane / 16 + 4 j][col = lane % 16]
    // (rows interleaved over the four lane groups): column 0 on lanes 0, 16,
    // 32, 48
    if (m == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = k + 4 * j;
            if (c < C) out[w * C + c] = base[i * 2 + 1] + acc[j];
        }
    }
}

template <int LPG>
__global__ __launch_bounds__(256) void k_dense_valu(int64_t nn, const int32_t *__restrict__ nodes, int C,
                                                    const double *__restrict__ rec_p,
                                                    const uint32_t *__restrict__ rec_z,
                                                    const uint32_t *__restrict__ off,
                                                    const uint32_t *__restrict__ cnt,
                                                    const double *__restrict__ base,
                                                    double *__restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= nn) return;
    const int64_t i = nodes[w];
    const uint64_t r0 = off[i];
    const uint32_t R = cnt[i];
    // LPG lanes per record group (one per chain), 64 / LPG groups
    const int c = lane % LPG, gidx = lane / LPG;
    double acc = 0.0;
    const uint32_t rot = (uint32_t)(c + 2) & 31u;
    for (uint32_t r = (uint32_t)gidx; r < R; r += 64 / LPG) {
        const uint32_t z = rec_z[r0 + r];
        const uint32_t hi = __builtin_amdgcn_alignbit(z, z, rot) & 0x40000000u;
        acc = __builtin_fma(__hiloint2double((int)hi, 0), rec_p[r0 + r], acc);
    }
#pragma unroll
    for (int o = LPG; o < 64; o <<= 1) acc += __shfl_xor(acc, o);
    if (gidx == 0 && c < C) out[w * C + c] = base[i * 2 + 1] + acc;
}

}  // namespace pdgd

extern "C" pdg_status pdg_dense_fields(pdg_ctx *ctx, int64_t n, const int32_t *d_nodes, int32_t method,
                                       double *d_out)
{
    pdg::CtxView v;
    pdg_status st = pdg::ctx_view(ctx, &v);
    if (st != PDG_OK) return st;
    if (v.QM != 2 || v.C > 16 || v.RP != 1 || v.ZW != 1)
        return pdg::report(ctx, PDG_EINVAL, "binary contexts with at most 16 chains only");
    if (v.phase != 1) return pdg::report(ctx, PDG_ESTATE, "fields are taken between the two phases");
    if (n < 0 || (n > 0 && (!d_nodes || !d_out)) || (method != 0 && method != 1))
        return pdg::report(ctx, PDG_EINVAL, "bad argument");
    if (n == 0) return PDG_OK;
    const unsigned blocks = (unsigned)((n + 3) / 4);
    if (method == 1)
        pdgd::k_dense_mfma<<<blocks, 256, 0, v.stream>>>(n, d_nodes, v.C, v.rec_p, v.rec_z, v.inc_off,
                                                          v.inc_cnt, v.base, d_out);
    else if (v.C <= 8)
        pdgd::k_dense_valu<8><<<blocks, 256, 0, v.stream>>>(n, d_nodes, v.C, v.rec_p, v.rec_z, v.inc_off,
                                                             v.inc_cnt, v.base, d_out);
    else
        pdgd::k_dense_valu<16><<<blocks, 256, 0, v.stream>>>(n, d_nodes, v.C, v.rec_p, v.rec_z,
                                                              v.inc_off, v.inc_cnt, v.base, d_out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return pdg::report(ctx, PDG_EHIP, hipGetErrorString(e));
    return PDG_OK;
}
