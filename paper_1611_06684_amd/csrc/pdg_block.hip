// Learned block proposal (blocking of Sec. 5.4) and its proposal network on
// the matrix cores.  C ABI in include/pdg_block.h.
//
// Layout: a binary H x W grid cut into 8 x 8 blocks; one wave per (block,
// chain) with lane p = block node p (row-major in the block), so a block's
// Metropolis-Hastings move is one wave's work and its sums are one wave
// reduction.  The network is three dense layers evaluated by one fused kernel
// per 64 rows (v_mfma_f32_16x16x32_bf16; activations stay in LDS); the
// backward pass uses a generic LDS-staged bf16 GEMM.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pdg.h"
#include "pdg_block.h"
#include "pdg_rng.hpp"
#include "pdg_view.hpp"

namespace pdgb {

using pdg::CtxView;
using pdg::Words;

constexpr uint32_t kPhaseBlock = 3u;
constexpr int BS = 8;           // block side
constexpr int NIN = PDG_MLP_IN, NH = PDG_MLP_HID, NOUT = PDG_MLP_OUT;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// Set-up.  Per node: f0 = lam(1) - lam(0) + the row / column terms of its
// inside edges (right, left, down, up, in that order) and the log odds ratios
// of its right and down inside edges.  Cut edges get their thresholds and
// fields from the decomposition's parameter blocks (pdg_decompose, q = 2:
// sign u64 @0, thr u32[2] @8, h f64 @16, c0 f64[2] @24).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_setup_nodes(int H, int W, const T *__restrict__ lphi, const T *__restrict__ lun,
                              double *__restrict__ f0, double *__restrict__ lint,
                              uint32_t *__restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)H * W) return;
    const int r = (int)(i / W), c = (int)(i % W);
    const int64_t nh = (int64_t)H * (W - 1);
    auto tab = [&](int64_t e, int a, int b) { return (double)lphi[e * 4 + a * 2 + b]; };
    double f = (double)lun[i * 2 + 1] - (double)lun[i * 2 + 0];
    bool ok = std::isfinite(f);
    double lr = 0.0, ld = 0.0;
    if (c + 1 < W && (c + 1) % BS != 0) {  // right edge, this node is src
        const int64_t e = (int64_t)r * (W - 1) + c;
        f += tab(e, 1, 0) - tab(e, 0, 0);
        lr = tab(e, 1, 1) + tab(e, 0, 0) - tab(e, 1, 0) - tab(e, 0, 1);
    }
    if (c > 0 && c % BS != 0) {  // left edge, this node is dst
        const int64_t e = (int64_t)r * (W - 1) + c - 1;
        f += tab(e, 0, 1) - tab(e, 0, 0);
    }
    if (r + 1 < H && (r + 1) % BS != 0) {  // down edge, src
        const int64_t e = nh + (int64_t)r * W + c;
        f += tab(e, 1, 0) - tab(e, 0, 0);
        ld = tab(e, 1, 1) + tab(e, 0, 0) - tab(e, 1, 0) - tab(e, 0, 1);
    }
    if (r > 0 && r % BS != 0) {  // up edge, dst
        const int64_t e = nh + (int64_t)(r - 1) * W + c;
        f += tab(e, 0, 1) - tab(e, 0, 0);
    }
    ok = ok && std::isfinite(f) && std::isfinite(lr) && std::isfinite(ld);
    f0[i] = f;
    lint[i * 2 + 0] = lr;
    lint[i * 2 + 1] = ld;
    if (!ok) *bad = 1u;
}

template <typename T>
__global__ void k_gather_tables(int64_t k, const int64_t *__restrict__ ids, const T *__restrict__ src,
                                T *__restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k * 4) dst[i] = src[ids[i / 4] * 4 + (i & 3)];
}

__global__ void k_setup_cut(int64_t ncut, const uint8_t *__restrict__ par, uint32_t *__restrict__ thr,
                            uint32_t *__restrict__ sign, double *__restrict__ fld)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ncut) return;
    const uint8_t *p = par + k * 40;
    const uint64_t sg = *reinterpret_cast<const uint64_t *>(p);
    const uint32_t *t = reinterpret_cast<const uint32_t *>(p + 8);
    const double h = *reinterpret_cast<const double *>(p + 16);
    const double *c0 = reinterpret_cast<const double *>(p + 24);
    thr[2 * k] = t[0];
    thr[2 * k + 1] = t[1];
    sign[k] = (uint32_t)(sg & 1u);
    fld[4 * k + 0] = c0[0];
    fld[4 * k + 1] = c0[1];
    fld[4 * k + 2] = 2.0 * h;
    fld[4 * k + 3] = 2.0 * fabs(h);
}

// ---------------------------------------------------------------------------
// Cut duals: thread per (cut edge, chain), the dual draw of Sec. 4 with the
// thresholds of the decomposition (theta = 1 iff U >= T(k), k = sigma (1 - 2y)
// + (1 - 2y'), T(+2) = T+, T(-2) = T-, T(0) = 2^23; compared on the word).
// ---------------------------------------------------------------------------
__global__ void k_cut_duals(int64_t ncut, int C, const int64_t *__restrict__ gid,
                            const int32_t *__restrict__ cnode, const uint32_t *__restrict__ thr,
                            const uint32_t *__restrict__ sign, const uint8_t *__restrict__ x,
                            uint8_t *__restrict__ theta, uint32_t s, pdg::RoundKeys rk)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ncut * C) return;
    const int64_t k = idx / C;
    const int c = (int)(idx - k * C);
    const uint64_t id = (uint64_t)gid[k] | (1ull << 63);
    const Words w = pdg::philox4x32_10((uint32_t)id, (uint32_t)(id >> 32),
                                       (kPhaseBlock << 30) | (uint32_t)(16 * c), s, rk);
    const int y = x[(int64_t)cnode[2 * k] * C + c], yp = x[(int64_t)cnode[2 * k + 1] * C + c];
    const int sg = sign[k] ? -1 : 1;
    const int kk = sg * (1 - 2 * y) + (1 - 2 * yp);
    const uint32_t W = w.w0;
    const bool th = kk > 0 ? (W > thr[2 * k]) : (kk < 0 ? (W >= thr[2 * k + 1]) : (W >= 0x80000000u));
    theta[idx] = th ? 1 : 0;
}

__global__ void k_scatter_theta(int64_t ncut, int C, const int64_t *__restrict__ gid,
                                const uint8_t *__restrict__ theta, uint8_t *__restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ncut * C) return;
    const int64_t k = idx / C;
    out[gid[k] * C + (idx - k * C)] = theta[idx];
}

struct BlockGeo {
    int W, nbc, C;
    const double *f0, *lint, *fld;
    const int32_t *slot;
    const uint8_t *theta;
};

__device__ __forceinline__ int64_t block_node(const BlockGeo &g, int64_t b, int p)
{
    const int64_t R0 = (b / g.nbc) * BS, C0 = (b % g.nbc) * BS;
    return (R0 + (p >> 3)) * g.W + C0 + (p & 7);
}

// The block kernels take one block and a tile of up to CT chains per
// work-group: the block's states and cut duals for the tile are staged in LDS
// (each node's chains are contiguous bytes in x, so the loads coalesce), then
// each wave takes the tile's chains in turn with lane = block node.
constexpr int CT = 64;

struct LaneSlots {
    // up to two cut edges of a block node (top / bottom, then left / right):
    // slot index, constant field, field per unit dual
    int t[2];
    double c0[2], hc[2];
};

__device__ __forceinline__ LaneSlots lane_slots(const BlockGeo &g, int64_t b, int p)
{
    LaneSlots s;
    const int row = p >> 3, col = p & 7;
    int n = 0;
    s.t[0] = s.t[1] = -1;
    s.c0[0] = s.c0[1] = s.hc[0] = s.hc[1] = 0.0;
    auto take = [&](int t, bool src) {
        const int k = g.slot[b * 32 + t];
        if (k >= 0) {
            s.t[n] = t;
            s.c0[n] = src ? g.fld[4 * k + 0] : g.fld[4 * k + 1];
            s.hc[n] = src ? g.fld[4 * k + 2] : g.fld[4 * k + 3];
            ++n;
        }
    };
    if (row == 0) take(col, false);
    if (row == 7) take(8 + col, true);
    if (col == 0) take(16 + row, false);
    if (col == 7) take(24 + row, true);
    return s;
}

// f of the lane's node for tile chain c: f0 plus its cut edges' fields in the
// order top, bottom, left, right.
__device__ __forceinline__ double tile_field(double f0, const LaneSlots &s, const uint8_t (*ts)[CT], int c)
{
    double f = f0;
#pragma unroll
    for (int j = 0; j < 2; ++j)
        if (s.t[j] >= 0) f += s.c0[j] + (double)ts[s.t[j]][c] * s.hc[j];
    return f;
}

__device__ __forceinline__ void stage_tile(const BlockGeo &g, int64_t b, int c0, int nc,
                                           const uint8_t *__restrict__ x, uint8_t (*xs)[CT],
                                           uint8_t (*ts)[CT])
{
    for (int q = threadIdx.x; q < 64 * CT; q += 256) {
        const int p = q / CT, c = q - p * CT;
        xs[p][c] = c < nc ? x[block_node(g, b, p) * g.C + c0 + c] : (uint8_t)0;
    }
    for (int q = threadIdx.x; q < 32 * CT; q += 256) {
        const int t = q / CT, c = q - t * CT;
        const int k = g.slot[b * 32 + t];
        ts[t][c] = (c < nc && k >= 0) ? g.theta[(int64_t)k * g.C + c0 + c] : (uint8_t)0;
    }
}

// Network inputs, targets and fields: grid (blocks, chain tiles).
__global__ __launch_bounds__(256) void k_inputs(BlockGeo g, const uint8_t *__restrict__ x,
                                                uint16_t *__restrict__ in, uint8_t *__restrict__ tgt,
                                                double *__restrict__ fout)
{
    __shared__ uint8_t xs[64][CT];
    __shared__ uint8_t ts[32][CT];
    const int64_t b = blockIdx.x;
    const int c0 = blockIdx.y * CT, nc = min(CT, g.C - c0);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    stage_tile(g, b, c0, nc, x, xs, ts);
    __syncthreads();
    const int64_t node = block_node(g, b, lane);
    const double f0 = g.f0[node];
    const LaneSlots sl = lane_slots(g, b, lane);
    for (int c = wv; c < nc; c += 4) {
        const int64_t row = b * g.C + c0 + c;
        const double f = tile_field(f0, sl, ts, c);
        in[row * NIN + lane] = bf16_bits((float)f);
        if (lane < 32) in[row * NIN + 64 + lane] = ts[lane][c] ? (uint16_t)0x3F80u : (uint16_t)0u;
        if (tgt) tgt[row * 64 + lane] = xs[lane][c];
        if (fout) fout[row * 64 + lane] = f;
    }
}

// Metropolis-Hastings move: grid (blocks, chain tiles); accepted proposals go
// into the staged tile, which is written back whole.
__global__ __launch_bounds__(256) void k_mh(BlockGeo g, uint8_t *__restrict__ x,
                                            const float *__restrict__ logits, uint32_t s,
                                            pdg::RoundKeys rk, unsigned long long *__restrict__ nacc,
                                            uint8_t *__restrict__ prop, uint8_t *__restrict__ accout,
                                            uint8_t *__restrict__ flagout)
{
    __shared__ uint8_t xs[64][CT];
    __shared__ uint8_t ts[32][CT];
    __shared__ uint32_t us[CT][66];  // the tile's 65 24-bit uniforms per chain
    __shared__ uint32_t nacc_ws[4];
    const int64_t b = blockIdx.x;
    const int c0 = blockIdx.y * CT, nc = min(CT, g.C - c0);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    stage_tile(g, b, c0, nc, x, xs, ts);
    // 13 generator calls per chain, each giving five uniforms (draw d: call
    // d / 5, slot d % 5), computed once for the tile
    for (int q = threadIdx.x; q < nc * 13; q += 256) {
        const int c = q / 13, k = q - 13 * c;
        const Words wd = pdg::philox4x32_10((uint32_t)b, (uint32_t)((uint64_t)b >> 32),
                                            (kPhaseBlock << 30) | (uint32_t)(16 * (c0 + c) + k), s, rk);
        const int d0 = 5 * k;
        us[c][d0] = wd.w0 >> 8;
        us[c][d0 + 1] = wd.w1 >> 8;
        us[c][d0 + 2] = wd.w2 >> 8;
        us[c][d0 + 3] = wd.w3 >> 8;
        if (d0 + 4 < 66) us[c][d0 + 4] = pdg::fifth_u24(wd);
    }
    __syncthreads();
    const int64_t node = block_node(g, b, lane);
    const double f0 = g.f0[node];
    const LaneSlots sl = lane_slots(g, b, lane);
    const int col = lane & 7, rowp = lane >> 3;
    const double lr = col < 7 ? g.lint[node * 2 + 0] : 0.0;
    const double ld = rowp < 7 ? g.lint[node * 2 + 1] : 0.0;
    uint32_t my_acc = 0;
    for (int c = wv; c < nc; c += 4) {
        const int64_t row = b * g.C + c0 + c;
        const int xv = xs[lane][c];
        const double f = tile_field(f0, sl, ts, c);
        const double l = (double)logits[row * 64 + lane];
        // proposal bit: u < sigmoid(l), the sigmoid in FP32, u exact in FP64
        const double u = ((double)us[c][lane] + 0.5) * 0x1p-24;
        const double p1 = (double)(1.0f / (1.0f + expf(-(float)l)));
        const int xp = u < p1 ? 1 : 0;
        bool flag = fabs(u - p1) < 1e-6;
        const uint32_t Uacc = us[c][64];
        const int xr = __shfl(xv, (lane + 1) & 63), xpr = __shfl(xp, (lane + 1) & 63);
        const int xd = __shfl(xv, (lane + 8) & 63), xpd = __shfl(xp, (lane + 8) & 63);
        double t = (double)(xp - xv) * (f - l);
        if (col < 7) t += lr * (double)(xp * xpr - xv * xr);
        if (rowp < 7) t += ld * (double)(xp * xpd - xv * xd);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o);
        const double lu = log(((double)Uacc + 0.5) * 0x1p-24);
        const bool acc = lu < t;
        flag = flag || fabs(lu - t) < 1e-9;
        if (acc) xs[lane][c] = (uint8_t)xp;
        const bool anyflag = __ballot(flag) != 0;
        if (prop) prop[row * 64 + lane] = (uint8_t)xp;
        if (lane == 0) {
            my_acc += acc ? 1u : 0u;
            if (accout) accout[row] = acc ? 1 : 0;
            if (flagout) flagout[row] = anyflag ? 1 : 0;
        }
    }
    if (lane == 0) nacc_ws[wv] = my_acc;
    __syncthreads();
    for (int q = threadIdx.x; q < 64 * CT; q += 256) {
        const int p = q / CT, c = q - p * CT;
        if (c < nc) x[block_node(g, b, p) * g.C + c0 + c] = xs[p][c];
    }
    if (threadIdx.x == 0) {
        const uint32_t tot = nacc_ws[0] + nacc_ws[1] + nacc_ws[2] + nacc_ws[3];
        if (tot) atomicAdd(nacc, (unsigned long long)tot);
    }
}

// ---------------------------------------------------------------------------
// Proposal network, forward: 64 rows per work-group of four waves.  Layers 1
// and 2: wave v computes output columns [64 v, 64 v + 64) for all 64 rows (4 x 4
// tiles of 16 x 16); layer 3: columns [16 v, 16 v + 16).  A operands (the
// activations) come from LDS, B operands (weights, [out][in], so eight
// consecutive k of one output column are 16 contiguous bytes) from global
// memory, where the 214 KB of weights stay in L2.
// ---------------------------------------------------------------------------
constexpr int TM = 64;
constexpr int XS = NIN + 8;  // LDS row strides in bf16 elements (16-byte multiples)
constexpr int HS = NH + 8;

template <int K, int SS>
__device__ __forceinline__ void dense_relu(const uint16_t *src, const uint16_t *__restrict__ Wt,
                                           const float *__restrict__ bias, uint16_t *dst, int wv,
                                           int lane)
{
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int lr = lane & 15, lk = 8 * (lane >> 4);
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 a[4], bb[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
            bb[nt] = *reinterpret_cast<const bf16x8 *>(Wt + (int64_t)(64 * wv + 16 * nt + lr) * K + k0 + lk);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            a[mt] = *reinterpret_cast<const bf16x8 *>(src + (16 * mt + lr) * SS + k0 + lk);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], bb[nt], acc[mt][nt], 0, 0, 0);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int col = 64 * wv + 16 * nt + lr;
        const float bv = bias[col];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * mt + 4 * (lane >> 4) + r;
                dst[row * HS + col] = bf16_bits(fmaxf(acc[mt][nt][r] + bv, 0.f));
            }
    }
}

__device__ __forceinline__ void tile_out(const uint16_t *hs, uint16_t *__restrict__ out, int64_t r0,
                                         int64_t rows, int tid)
{
    // 64 rows x 256 bf16 = 2048 chunks of 16 bytes
    for (int q = tid; q < TM * (NH / 8); q += 256) {
        const int r = q / (NH / 8), ch = q - r * (NH / 8);
        if (r0 + r < rows)
            *reinterpret_cast<uint4 *>(out + (r0 + r) * NH + ch * 8) =
                *reinterpret_cast<const uint4 *>(hs + r * HS + ch * 8);
    }
}

__global__ __launch_bounds__(256) void k_mlp_fwd(const uint16_t *__restrict__ wbf,
                                                 const float *__restrict__ w32, int64_t rows,
                                                 const uint16_t *__restrict__ in,
                                                 float *__restrict__ logits,
                                                 uint16_t *__restrict__ h1out,
                                                 uint16_t *__restrict__ h2out)
{
    __shared__ __align__(16) uint16_t xs[TM * XS];
    __shared__ __align__(16) uint16_t h1[TM * HS];
    __shared__ __align__(16) uint16_t h2[TM * HS];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * TM;
    for (int q = tid; q < TM * (NIN / 8); q += 256) {
        const int r = q / (NIN / 8), ch = q - r * (NIN / 8);
        uint4 v = make_uint4(0, 0, 0, 0);
        if (r0 + r < rows) v = *reinterpret_cast<const uint4 *>(in + (r0 + r) * NIN + ch * 8);
        *reinterpret_cast<uint4 *>(xs + r * XS + ch * 8) = v;
    }
    __syncthreads();
    dense_relu<NIN, XS>(xs, wbf + PDG_MLP_OFF_W1, w32 + PDG_MLP_OFF_B1, h1, wv, lane);
    __syncthreads();
    if (h1out) tile_out(h1, h1out, r0, rows, tid);
    dense_relu<NH, HS>(h1, wbf + PDG_MLP_OFF_W2, w32 + PDG_MLP_OFF_B2, h2, wv, lane);
    __syncthreads();
    if (h2out) tile_out(h2, h2out, r0, rows, tid);
    // layer 3: columns [16 wv, 16 wv + 16), residual = the row's input fields
    const int lr = lane & 15, lk = 8 * (lane >> 4);
    f32x4 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t *W3 = wbf + PDG_MLP_OFF_W3;
    for (int k0 = 0; k0 < NH; k0 += 32) {
        const bf16x8 bb = *reinterpret_cast<const bf16x8 *>(W3 + (int64_t)(16 * wv + lr) * NH + k0 + lk);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(h2 + (16 * mt + lr) * HS + k0 + lk);
            acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc[mt], 0, 0, 0);
        }
    }
    const int col = 16 * wv + lr;
    const float bv = w32[PDG_MLP_OFF_B3 + col];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * mt + 4 * (lane >> 4) + r;
            if (r0 + row < rows)
                logits[(r0 + row) * NOUT + col] = acc[mt][r] + bv + bf16_float(xs[row * XS + col]);
        }
}

// ---------------------------------------------------------------------------
// Backward pass.  dl = (sigmoid(l) - t) / R rounded to BF16, with the loss;
// generic GEMM C = A B (bf16 in, FP32 accumulate; 64 x 64 tiles, k steps of 32
// staged through LDS; A either k-contiguous [M][K] or m-contiguous [K][M], B
// n-contiguous [K][N]); deterministic two-pass column sums for the biases.
// ---------------------------------------------------------------------------
__global__ void k_bce_grad(int64_t rows, const float *__restrict__ logits, const uint8_t *__restrict__ tgt,
                           uint16_t *__restrict__ dL, double *__restrict__ loss)
{
    __shared__ double red[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double lv = 0.0;
    if (i < rows * NOUT) {
        const float l = logits[i];
        const float t = (float)tgt[i];
        const float sg = 1.0f / (1.0f + expf(-l));
        dL[i] = bf16_bits((sg - t) / (float)rows);
        lv = (double)(fmaxf(l, 0.f) + log1pf(expf(-fabsf(l))) - t * l);
    }
    if (loss) {
        for (int o = 32; o >= 1; o >>= 1) lv += __shfl_xor(lv, o);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lv;
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(loss, (red[0] + red[1] + red[2] + red[3]) / (double)rows);
    }
}

enum { EPI_F32 = 0, EPI_MASK_BF16 = 1 };

template <bool A_MCONTIG, int EPI>
__global__ __launch_bounds__(256) void k_gemm(int64_t M, int64_t N, int64_t K,
                                              const uint16_t *__restrict__ A, int64_t lda,
                                              const uint16_t *__restrict__ B, int64_t ldb,
                                              void *__restrict__ out, int64_t ldo,
                                              const uint16_t *__restrict__ mask)
{
    constexpr int LS = 32 + 8;  // LDS row stride (bf16)
    __shared__ __align__(16) uint16_t As[64 * LS];
    __shared__ __align__(16) uint16_t Bs[64 * LS];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv >> 1, wn = wv & 1;
    const int64_t m0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int lr = lane & 15, lk = 8 * (lane >> 4);
    for (int64_t k0 = 0; k0 < K; k0 += 32) {
        // A tile [64 m][32 k]: 256 chunks of 8 elements
        if (!A_MCONTIG) {  // A[m * lda + k]
            const int m = tid >> 2, kc = (tid & 3) * 8;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (m0 + m < M && k0 + kc < K) v = *reinterpret_cast<const uint4 *>(A + (m0 + m) * lda + k0 + kc);
            *reinterpret_cast<uint4 *>(As + m * LS + kc) = v;
        } else {  // A[k * lda + m]
            const int k = tid >> 3, mc = (tid & 7) * 8;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (k0 + k < K && m0 + mc < M) v = *reinterpret_cast<const uint4 *>(A + (k0 + k) * lda + m0 + mc);
            const uint16_t *e = reinterpret_cast<const uint16_t *>(&v);
#pragma unroll
            for (int j = 0; j < 8; ++j) As[(mc + j) * LS + k] = e[j];
        }
        {  // B tile: B[k * ldb + n] -> Bs[n][k]
            const int k = tid >> 3, nc = (tid & 7) * 8;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (k0 + k < K && n0 + nc < N) v = *reinterpret_cast<const uint4 *>(B + (k0 + k) * ldb + n0 + nc);
            const uint16_t *e = reinterpret_cast<const uint16_t *>(&v);
#pragma unroll
            for (int j = 0; j < 8; ++j) Bs[(nc + j) * LS + k] = e[j];
        }
        __syncthreads();
        bf16x8 a[2], bb[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            a[i] = *reinterpret_cast<const bf16x8 *>(As + (32 * wm + 16 * i + lr) * LS + lk);
            bb[i] = *reinterpret_cast<const bf16x8 *>(Bs + (32 * wn + 16 * i + lr) * LS + lk);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bb[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + 32 * wm + 16 * i + 4 * (lane >> 4) + r;
                const int64_t col = n0 + 32 * wn + 16 * j + lr;
                if (row < M && col < N) {
                    const float v = acc[i][j][r];
                    if (EPI == EPI_F32)
                        static_cast<float *>(out)[row * ldo + col] = v;
                    else
                        static_cast<uint16_t *>(out)[row * ldo + col] =
                            bf16_bits(bf16_float(mask[row * ldo + col]) > 0.f ? v : 0.f);
                }
            }
}

// Column sums of a bf16 [R][N] matrix: part[chunk][n] over 256-row chunks, then
// out[n] = sum of the chunks in order.
__global__ __launch_bounds__(256) void k_colsum_part(int64_t R, int N, const uint16_t *__restrict__ D,
                                                     float *__restrict__ part)
{
    __shared__ float red[4][64];
    const int cx = threadIdx.x & 63, ry = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + cx;
    const int64_t r0 = (int64_t)blockIdx.y * 256;
    float s = 0.f;
    if (n < N)
        for (int64_t r = r0 + ry; r < std::min<int64_t>(r0 + 256, R); r += 4) s += bf16_float(D[r * N + n]);
    red[ry][cx] = s;
    __syncthreads();
    if (ry == 0 && n < N) part[(int64_t)blockIdx.y * N + n] = (red[0][cx] + red[1][cx]) + (red[2][cx] + red[3][cx]);
}

__global__ void k_colsum_fin(int64_t chunks, int N, const float *__restrict__ part, float *__restrict__ out)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int64_t k = 0; k < chunks; ++k) s += part[k * N + n];
    out[n] = s;
}

__global__ void k_adam(int64_t np, float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2,
                       uint16_t *__restrict__ wbf)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    w[i] = wi;
    wbf[i] = bf16_bits(wi);
}

__global__ void k_fill_f64(double *p, double v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

}  // namespace pdgb

using namespace pdgb;

struct pdg_blk {
    pdg_ctx *ctx = nullptr;
    int32_t H = 0, W = 0, nbr = 0, nbc = 0, C = 0;
    int64_t nb = 0, n = 0, m = 0, ncut = 0;
    int64_t s = 0, proposed = 0;
    double *d_f0 = nullptr, *d_lint = nullptr, *d_fld = nullptr;
    int32_t *d_slot = nullptr, *d_cnode = nullptr;
    int64_t *d_cgid = nullptr;
    uint32_t *d_thr = nullptr, *d_sign = nullptr, *d_flag = nullptr;
    uint8_t *d_theta = nullptr;
    unsigned long long *d_nacc = nullptr;
};

namespace {

pdg_status blk_fail(pdg_blk *b, pdg_status code, const std::string &msg)
{
    return pdg::report(b ? b->ctx : nullptr, code, msg);
}

#define BLK_HIP(b, expr)                                                                         \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return blk_fail((b), PDG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define MLP_HIP(expr)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return pdg::report(nullptr, PDG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

void blk_free(pdg_blk *b)
{
    void *ps[] = {b->d_f0, b->d_lint, b->d_fld, b->d_slot, b->d_cnode, b->d_cgid,
                  b->d_thr, b->d_sign, b->d_flag, b->d_theta, b->d_nacc};
    for (void *p : ps)
        if (p) (void)hipFree(p);
}

template <typename T>
pdg_status setup_tables(pdg_blk *b, const CtxView &v, const void *d_log_phi, const void *d_log_unary,
                        const int64_t *d_ids, void *d_tmp)
{
    const int64_t n = b->n;
    k_setup_nodes<T><<<(unsigned)cdiv(n, 256), 256, 0, v.stream>>>(
        b->H, b->W, static_cast<const T *>(d_log_phi), static_cast<const T *>(d_log_unary), b->d_f0,
        b->d_lint, b->d_flag);
    BLK_HIP(b, hipGetLastError());
    if (b->ncut) {
        k_gather_tables<T><<<(unsigned)cdiv(b->ncut * 4, 256), 256, 0, v.stream>>>(
            b->ncut, d_ids, static_cast<const T *>(d_log_phi), static_cast<T *>(d_tmp));
        BLK_HIP(b, hipGetLastError());
    }
    return PDG_OK;
}

}  // namespace

extern "C" {

pdg_status pdg_blk_create(pdg_ctx *ctx, int32_t H, int32_t W, const void *d_log_phi,
                          const void *d_log_unary, pdg_blk **out)
{
    if (!out) return pdg::report(ctx, PDG_EINVAL, "null argument");
    *out = nullptr;
    CtxView v;
    pdg_status st = pdg::ctx_view(ctx, &v);
    if (st != PDG_OK) return st;
    if (!d_log_phi || !d_log_unary) return pdg::report(ctx, PDG_EINVAL, "null pointer");
    if (H < 8 || W < 8 || H % 8 || W % 8) return pdg::report(ctx, PDG_EINVAL, "H and W must be multiples of 8");
    if (v.QM != 2 || v.n != (int64_t)H * W)
        return pdg::report(ctx, PDG_EINVAL, "the context must hold H * W binary nodes (q_max 2)");
    if ((int64_t)H * W >= (1ll << 31) || v.C > (1 << 26))
        return pdg::report(ctx, PDG_EINVAL, "grid too large");
    pdg_blk *b = new (std::nothrow) pdg_blk();
    if (!b) return pdg::report(ctx, PDG_ENOMEM, "host allocation failed");
    b->ctx = ctx;
    b->H = H;
    b->W = W;
    b->nbr = H / 8;
    b->nbc = W / 8;
    b->nb = (int64_t)b->nbr * b->nbc;
    b->n = (int64_t)H * W;
    b->m = (int64_t)H * (W - 1) + (int64_t)(H - 1) * W;
    b->C = v.C;
    // cut edges (grid order) and each block's 32 boundary slots
    const int64_t nh = (int64_t)H * (W - 1);
    std::vector<int64_t> gid;
    std::vector<int32_t> cnode;
    for (int r = 0; r < H; ++r)
        for (int c = 0; c + 1 < W; ++c)
            if ((c + 1) % 8 == 0) {
                gid.push_back((int64_t)r * (W - 1) + c);
                cnode.push_back(r * W + c);
                cnode.push_back(r * W + c + 1);
            }
    for (int r = 0; r + 1 < H; ++r)
        if ((r + 1) % 8 == 0)
            for (int c = 0; c < W; ++c) {
                gid.push_back(nh + (int64_t)r * W + c);
                cnode.push_back(r * W + c);
                cnode.push_back((r + 1) * W + c);
            }
    b->ncut = (int64_t)gid.size();
    std::vector<int64_t> index_of(b->m, -1);
    for (int64_t k = 0; k < b->ncut; ++k) index_of[gid[k]] = k;
    std::vector<int32_t> slot(b->nb * 32, -1);
    for (int64_t bl = 0; bl < b->nb; ++bl) {
        const int R0 = (int)(bl / b->nbc) * 8, C0 = (int)(bl % b->nbc) * 8;
        for (int k = 0; k < 8; ++k) {
            if (R0 > 0) slot[bl * 32 + k] = (int32_t)index_of[nh + (int64_t)(R0 - 1) * W + C0 + k];
            if (R0 + 8 < H) slot[bl * 32 + 8 + k] = (int32_t)index_of[nh + (int64_t)(R0 + 7) * W + C0 + k];
            if (C0 > 0) slot[bl * 32 + 16 + k] = (int32_t)index_of[(int64_t)(R0 + k) * (W - 1) + C0 - 1];
            if (C0 + 8 < W) slot[bl * 32 + 24 + k] = (int32_t)index_of[(int64_t)(R0 + k) * (W - 1) + C0 + 7];
        }
    }
    auto fail_free = [&](pdg_status code, const std::string &msg) {
        blk_free(b);
        delete b;
        return pdg::report(ctx, code, msg);
    };
#define BLK_ALLOC(ptr, bytes)                                                                    \
    if (hipMalloc((void **)&(ptr), std::max<int64_t>((bytes), 8)) != hipSuccess)                \
        return fail_free(PDG_ENOMEM, "hipMalloc failed");
    const int64_t nc = std::max<int64_t>(b->ncut, 1);
    BLK_ALLOC(b->d_f0, b->n * 8);
    BLK_ALLOC(b->d_lint, b->n * 16);
    BLK_ALLOC(b->d_fld, nc * 32);
    BLK_ALLOC(b->d_slot, b->nb * 32 * 4);
    BLK_ALLOC(b->d_cnode, nc * 8);
    BLK_ALLOC(b->d_cgid, nc * 8);
    BLK_ALLOC(b->d_thr, nc * 8);
    BLK_ALLOC(b->d_sign, nc * 4);
    BLK_ALLOC(b->d_flag, 4);
    BLK_ALLOC(b->d_theta, nc * b->C);
    BLK_ALLOC(b->d_nacc, 8);
    const bool f64 = v.precision == PDG_PRECISION_F64;
    const int64_t esz = f64 ? 8 : 4;
    uint8_t *d_par = nullptr;
    void *d_tmp = nullptr;
    int32_t *d_q2 = nullptr;
    BLK_ALLOC(d_par, nc * 40);
    if (hipMalloc(&d_tmp, nc * 4 * esz) != hipSuccess || hipMalloc((void **)&d_q2, nc * 4) != hipSuccess) {
        (void)hipFree(d_par);
        (void)hipFree(d_tmp);
        return fail_free(PDG_ENOMEM, "hipMalloc failed");
    }
    auto cleanup = [&]() {
        (void)hipFree(d_par);
        (void)hipFree(d_tmp);
        (void)hipFree(d_q2);
    };
    std::vector<int32_t> twos(nc, 2);
    hipError_t e = hipMemcpyAsync(b->d_slot, slot.data(), b->nb * 32 * 4, hipMemcpyHostToDevice, v.stream);
    if (e == hipSuccess && b->ncut)
        e = hipMemcpyAsync(b->d_cnode, cnode.data(), b->ncut * 8, hipMemcpyHostToDevice, v.stream);
    if (e == hipSuccess && b->ncut)
        e = hipMemcpyAsync(b->d_cgid, gid.data(), b->ncut * 8, hipMemcpyHostToDevice, v.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_q2, twos.data(), nc * 4, hipMemcpyHostToDevice, v.stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_flag, 0, 4, v.stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_nacc, 0, 8, v.stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_theta, 0, nc * b->C, v.stream);
    if (e != hipSuccess) {
        cleanup();
        return fail_free(PDG_EHIP, std::string("set-up copies: ") + hipGetErrorString(e));
    }
    st = f64 ? setup_tables<double>(b, v, d_log_phi, d_log_unary, b->d_cgid, d_tmp)
             : setup_tables<float>(b, v, d_log_phi, d_log_unary, b->d_cgid, d_tmp);
    if (st == PDG_OK && b->ncut) {
        st = pdg_decompose(b->ncut, 2, d_q2, d_q2, d_tmp, v.precision, d_par, v.stream);
        if (st != PDG_OK) st = pdg::report(ctx, st, std::string("cut edges: ") + pdg_last_error(nullptr));
    }
    if (st == PDG_OK && b->ncut) {
        k_setup_cut<<<(unsigned)cdiv(b->ncut, 256), 256, 0, v.stream>>>(b->ncut, d_par, b->d_thr,
                                                                        b->d_sign, b->d_fld);
        e = hipGetLastError();
        if (e != hipSuccess) st = pdg::report(ctx, PDG_EHIP, hipGetErrorString(e));
    }
    uint32_t bad = 0;
    if (st == PDG_OK) {
        e = hipMemcpyAsync(&bad, b->d_flag, 4, hipMemcpyDeviceToHost, v.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(v.stream);
        if (e != hipSuccess) st = pdg::report(ctx, PDG_EHIP, hipGetErrorString(e));
        else if (bad) st = pdg::report(ctx, PDG_ENONPOS, "non-finite log factor or unary entry");
    }
    cleanup();
    if (st != PDG_OK) {
        blk_free(b);
        delete b;
        return st;
    }
    *out = b;
    return PDG_OK;
#undef BLK_ALLOC
}

pdg_status pdg_blk_destroy(pdg_blk *b)
{
    if (!b) return PDG_OK;
    blk_free(b);
    delete b;
    return PDG_OK;
}

static pdg_status blk_view(pdg_blk *b, CtxView *v, bool between_sweeps)
{
    if (!b) return pdg::report(nullptr, PDG_EINVAL, "null block object");
    pdg_status st = pdg::ctx_view(b->ctx, v);
    if (st != PDG_OK) return st;
    if (between_sweeps && v->phase != 0)
        return blk_fail(b, PDG_ESTATE, "block moves run between sweeps");
    return PDG_OK;
}

static BlockGeo geo(const pdg_blk *b)
{
    return BlockGeo{b->W, b->nbc, b->C, b->d_f0, b->d_lint, b->d_fld, b->d_slot, b->d_theta};
}

pdg_status pdg_blk_cut_duals(pdg_blk *b)
{
    CtxView v;
    pdg_status st = blk_view(b, &v, true);
    if (st != PDG_OK) return st;
    if (b->s + 1 >= (1ll << 32)) return blk_fail(b, PDG_ECAPACITY, "step counter exhausted");
    b->s += 1;
    if (b->ncut) {
        k_cut_duals<<<(unsigned)cdiv(b->ncut * b->C, 256), 256, 0, v.stream>>>(
            b->ncut, b->C, b->d_cgid, b->d_cnode, b->d_thr, b->d_sign, v.d_x, b->d_theta, (uint32_t)b->s,
            pdg::make_round_keys(v.seed));
        BLK_HIP(b, hipGetLastError());
    }
    return PDG_OK;
}

pdg_status pdg_blk_inputs(pdg_blk *b, uint16_t *d_in, uint8_t *d_target, double *d_fields)
{
    CtxView v;
    pdg_status st = blk_view(b, &v, true);
    if (st != PDG_OK) return st;
    if (!d_in) return blk_fail(b, PDG_EINVAL, "null input buffer");
    k_inputs<<<dim3((unsigned)b->nb, (unsigned)cdiv(b->C, CT)), 256, 0, v.stream>>>(geo(b), v.d_x, d_in,
                                                                                   d_target, d_fields);
    BLK_HIP(b, hipGetLastError());
    return PDG_OK;
}

pdg_status pdg_blk_mh(pdg_blk *b, const float *d_logits, uint8_t *d_prop, uint8_t *d_acc, uint8_t *d_flag)
{
    CtxView v;
    pdg_status st = blk_view(b, &v, true);
    if (st != PDG_OK) return st;
    if (!d_logits) return blk_fail(b, PDG_EINVAL, "null logits");
    if (b->s == 0) return blk_fail(b, PDG_ESTATE, "pdg_blk_cut_duals first");
    k_mh<<<dim3((unsigned)b->nb, (unsigned)cdiv(b->C, CT)), 256, 0, v.stream>>>(
        geo(b), v.d_x, d_logits, (uint32_t)b->s, pdg::make_round_keys(v.seed), b->d_nacc, d_prop, d_acc,
        d_flag);
    BLK_HIP(b, hipGetLastError());
    b->proposed += b->nb * b->C;
    return PDG_OK;
}

pdg_status pdg_blk_get_cut_duals(pdg_blk *b, uint8_t *d_theta)
{
    CtxView v;
    pdg_status st = blk_view(b, &v, false);
    if (st != PDG_OK) return st;
    if (!d_theta) return blk_fail(b, PDG_EINVAL, "null output");
    BLK_HIP(b, hipMemsetAsync(d_theta, 0, b->m * b->C, v.stream));
    if (b->ncut) {
        k_scatter_theta<<<(unsigned)cdiv(b->ncut * b->C, 256), 256, 0, v.stream>>>(b->ncut, b->C, b->d_cgid,
                                                                                   b->d_theta, d_theta);
        BLK_HIP(b, hipGetLastError());
    }
    BLK_HIP(b, hipStreamSynchronize(v.stream));
    return PDG_OK;
}

pdg_status pdg_blk_info(pdg_blk *b, int64_t *h_step, int64_t *h_blocks, int64_t *h_accepted,
                        int64_t *h_proposed)
{
    CtxView v;
    pdg_status st = blk_view(b, &v, false);
    if (st != PDG_OK) return st;
    unsigned long long acc = 0;
    if (h_accepted) {
        BLK_HIP(b, hipMemcpyAsync(&acc, b->d_nacc, 8, hipMemcpyDeviceToHost, v.stream));
        BLK_HIP(b, hipStreamSynchronize(v.stream));
        *h_accepted = (int64_t)acc;
    }
    if (h_step) *h_step = b->s;
    if (h_blocks) *h_blocks = b->nb;
    if (h_proposed) *h_proposed = b->proposed;
    return PDG_OK;
}

pdg_status pdg_blk_set_step(pdg_blk *b, int64_t s)
{
    if (!b) return pdg::report(nullptr, PDG_EINVAL, "null block object");
    if (s < 0 || s >= (1ll << 32)) return blk_fail(b, PDG_EINVAL, "step out of range");
    b->s = s;
    return PDG_OK;
}

pdg_status pdg_mlp_forward(const uint16_t *d_wbf, const float *d_w32, int64_t rows, const uint16_t *d_in,
                           float *d_logits, uint16_t *d_h1, uint16_t *d_h2, void *stream)
{
    if (rows < 0) return pdg::report(nullptr, PDG_EINVAL, "rows < 0");
    if (rows == 0) return PDG_OK;
    if (!d_wbf || !d_w32 || !d_in || !d_logits) return pdg::report(nullptr, PDG_EINVAL, "null pointer");
    if (((uintptr_t)d_wbf | (uintptr_t)d_in | (uintptr_t)d_h1 | (uintptr_t)d_h2) & 15)
        return pdg::report(nullptr, PDG_EINVAL, "BF16 buffers must be 16-byte aligned");
    if (rows > (1ll << 40)) return pdg::report(nullptr, PDG_EINVAL, "too many rows");
    k_mlp_fwd<<<(unsigned)cdiv(rows, TM), 256, 0, (hipStream_t)stream>>>(d_wbf, d_w32, rows, d_in, d_logits,
                                                                         d_h1, d_h2);
    MLP_HIP(hipGetLastError());
    return PDG_OK;
}

static int64_t a256(int64_t x) { return (x + 255) / 256 * 256; }

pdg_status pdg_mlp_backward_workspace(int64_t rows, int64_t *h_bytes)
{
    if (rows < 0 || !h_bytes) return pdg::report(nullptr, PDG_EINVAL, "bad argument");
    *h_bytes = a256(rows * NOUT * 2) + 2 * a256(rows * NH * 2) + a256(cdiv(rows, 256) * NH * 4);
    return PDG_OK;
}

pdg_status pdg_mlp_backward(const uint16_t *d_wbf, int64_t rows, const uint16_t *d_in, const uint16_t *d_h1,
                            const uint16_t *d_h2, const float *d_logits, const uint8_t *d_target,
                            float *d_grad, double *d_loss, void *d_work, int64_t work_bytes, void *stream)
{
    if (rows <= 0) return pdg::report(nullptr, PDG_EINVAL, "rows must be >= 1");
    if (!d_wbf || !d_in || !d_h1 || !d_h2 || !d_logits || !d_target || !d_grad || !d_work)
        return pdg::report(nullptr, PDG_EINVAL, "null pointer");
    if (((uintptr_t)d_wbf | (uintptr_t)d_in | (uintptr_t)d_h1 | (uintptr_t)d_h2 | (uintptr_t)d_work) & 15)
        return pdg::report(nullptr, PDG_EINVAL, "buffers must be 16-byte aligned");
    int64_t need = 0;
    pdg_mlp_backward_workspace(rows, &need);
    if (work_bytes < need) return pdg::report(nullptr, PDG_EINVAL, "workspace too small");
    const hipStream_t st = (hipStream_t)stream;
    char *w = static_cast<char *>(d_work);
    uint16_t *dL = reinterpret_cast<uint16_t *>(w);
    uint16_t *dH2 = reinterpret_cast<uint16_t *>(w + a256(rows * NOUT * 2));
    uint16_t *dH1 = reinterpret_cast<uint16_t *>(w + a256(rows * NOUT * 2) + a256(rows * NH * 2));
    float *part = reinterpret_cast<float *>(w + a256(rows * NOUT * 2) + 2 * a256(rows * NH * 2));
    const int64_t chunks = cdiv(rows, 256);
    if (d_loss) k_fill_f64<<<1, 64, 0, st>>>(d_loss, 0.0);
    k_bce_grad<<<(unsigned)cdiv(rows * NOUT, 256), 256, 0, st>>>(rows, d_logits, d_target, dL, d_loss);
    // dH2 = (dL W3) masked by H2 > 0; dH1 = (dH2 W2) masked by H1 > 0
    k_gemm<false, EPI_MASK_BF16><<<dim3(NH / 64, (unsigned)cdiv(rows, 64)), 256, 0, st>>>(
        rows, NH, NOUT, dL, NOUT, d_wbf + PDG_MLP_OFF_W3, NH, dH2, NH, d_h2);
    k_gemm<false, EPI_MASK_BF16><<<dim3(NH / 64, (unsigned)cdiv(rows, 64)), 256, 0, st>>>(
        rows, NH, NH, dH2, NH, d_wbf + PDG_MLP_OFF_W2, NH, dH1, NH, d_h1);
    // weight gradients: dW3 = dL^T H2, dW2 = dH2^T H1, dW1 = dH1^T X
    k_gemm<true, EPI_F32><<<dim3(NH / 64, NOUT / 64), 256, 0, st>>>(NOUT, NH, rows, dL, NOUT, d_h2, NH,
                                                                     d_grad + PDG_MLP_OFF_W3, NH, nullptr);
    k_gemm<true, EPI_F32><<<dim3(NH / 64, NH / 64), 256, 0, st>>>(NH, NH, rows, dH2, NH, d_h1, NH,
                                                                   d_grad + PDG_MLP_OFF_W2, NH, nullptr);
    k_gemm<true, EPI_F32><<<dim3((unsigned)cdiv(NIN, 64), NH / 64), 256, 0, st>>>(
        NH, NIN, rows, dH1, NH, d_in, NIN, d_grad + PDG_MLP_OFF_W1, NIN, nullptr);
    // bias gradients
    const struct { const uint16_t *D; int N; int off; } cs[3] = {
        {dL, NOUT, PDG_MLP_OFF_B3}, {dH2, NH, PDG_MLP_OFF_B2}, {dH1, NH, PDG_MLP_OFF_B1}};
    for (const auto &c : cs) {
        k_colsum_part<<<dim3((unsigned)cdiv(c.N, 64), (unsigned)chunks), 256, 0, st>>>(rows, c.N, c.D, part);
        k_colsum_fin<<<(unsigned)cdiv(c.N, 256), 256, 0, st>>>(chunks, c.N, part, d_grad + c.off);
    }
    MLP_HIP(hipGetLastError());
    return PDG_OK;
}

pdg_status pdg_mlp_adam(float *d_w, const float *d_g, float *d_m, float *d_v, int64_t step, float lr,
                        float beta1, float beta2, float eps, uint16_t *d_wbf, void *stream)
{
    if (!d_w || !d_g || !d_m || !d_v || !d_wbf) return pdg::report(nullptr, PDG_EINVAL, "null pointer");
    if (step < 1) return pdg::report(nullptr, PDG_EINVAL, "step must be >= 1");
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
    k_adam<<<(unsigned)cdiv(PDG_MLP_PARAMS, 256), 256, 0, (hipStream_t)stream>>>(
        PDG_MLP_PARAMS, d_w, d_g, d_m, d_v, lr, beta1, beta2, eps, c1, c2, d_wbf);
    MLP_HIP(hipGetLastError());
    return PDG_OK;
}

}  // extern "C"
