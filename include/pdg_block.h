/*
 * pdg_block.h -- C ABI of the learned block proposal: blocked sampling with
 * respect to the duals of the edges between blocks (Sec. 5.4 Blocking of
 * Mescheder, Nowozin, Geiger, arXiv:1611.06684), where the exact draw of a
 * block given those duals is replaced by a Metropolis-Hastings move with a
 * learned independence proposal.  Built into libpdg.so.
 *
 * Model.  A binary H x W grid (H, W multiples of 8; node r*W + c; edges in the
 * order horizontal (r,c)-(r,c+1) row-major, then vertical (r,c)-(r+1,c)
 * row-major, src = left/top end) cut into 8 x 8 blocks (block (R, C') =
 * R*(W/8) + C', nodes row-major inside).  Duals are kept only on the edges that
 * cross blocks ("cut" edges; Sec. 5.4's theta_1).  Given them the blocks are
 * independent: p(x_B | theta_1) is proportional to
 * exp(sum_i f_i x_i + sum_{e inside B} l_e x_src x_dst), with f_i the node's
 * log-odds from its unary, the inside edges' row/column terms and, per cut
 * edge, the field of the Theorem's decomposition given theta_e (Sec. 4.1,
 * 4.2), and l_e an inside edge's log odds ratio.
 *
 * One learned step: pdg_blk_cut_duals (theta_e ~ p(theta_e | x) for every cut
 * edge and chain), pdg_blk_inputs (the proposal network's input rows),
 * pdg_mlp_forward (64 logits per block and chain), pdg_blk_mh (x'_B ~
 * prod_i Bernoulli(sigmoid(l_i)); accept with probability
 * min(1, exp(sum_i (x'_i - x_i)(f_i - l_i) + sum_e l_e (x'_src x'_dst -
 * x_src x_dst)))).  The plain sweep of the context (pdg_sweep) is the
 * fallback move; each leaves p(x) invariant.
 *
 * Generator: Philox4x32-10 with the context's seed, phase 3 and the block
 * object's step counter s: cut edge e draws word 0 of call (2^63 + e, sub 16c);
 * block b, chain c draws 65 uniforms from calls (b, sub 16c + k), k = 0..12,
 * five 24-bit uniforms per call as the dual phase takes them (draw d: call
 * d / 5, slot d mod 5; d < 64 the proposal bit of block node d, d = 64 the
 * acceptance).
 *
 * Network rows are block-major, chain-minor (row = b * C + c).  Input row:
 * 64 BF16 fields f (FP64 rounded to nearest even) then 32 boundary dual bits
 * (top side columns 0..7, bottom, left rows 0..7, right; 0 where the grid has
 * no edge).  Network: 96 -> 256 -> 256 -> 64, ReLU, BF16 weights and
 * activations on the matrix cores with FP32 accumulation; logits = last
 * layer + bias + the row's 64 input fields (residual).
 *
 * Conventions as in pdg.h: d_* device pointers owned by the caller, work on
 * the given stream (the context's for pdg_blk_*), PDG_* status codes.
 */
#ifndef PDG_BLOCK_H
#define PDG_BLOCK_H

#include <stdint.h>

#include "pdg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Packed network parameters: one array of PDG_MLP_PARAMS values, W1 [256][96],
 * b1 [256], W2 [256][256], b2 [256], W3 [64][256], b3 [64] at these offsets
 * (weights row-major [out][in]).  The FP32 array holds every parameter; the
 * BF16 array (same offsets, uint16 bit patterns) holds the weight matrices the
 * matrix cores read (its bias entries are unused). */
enum {
    PDG_MLP_IN = 96, PDG_MLP_HID = 256, PDG_MLP_OUT = 64,
    PDG_MLP_OFF_W1 = 0, PDG_MLP_OFF_B1 = 24576, PDG_MLP_OFF_W2 = 24832,
    PDG_MLP_OFF_B2 = 90368, PDG_MLP_OFF_W3 = 90624, PDG_MLP_OFF_B3 = 107008,
    PDG_MLP_PARAMS = 107072
};

typedef struct pdg_blk pdg_blk;

/* Blocking of the context's grid.  ctx: q_max 2, every q_i = 2, n = H W, C
 * chains; d_log_phi: [m][2][2] log tables of the grid's m = H(W-1) + (H-1)W
 * edges in the order above, d_log_unary: [n][2], in the context's precision
 * (they are decomposed here; the context's own edges are not read).
 * Non-finite entries give PDG_ENONPOS; sizes not multiples of 8, q_max != 2 or
 * n != H W give PDG_EINVAL.  Synchronizes the stream. */
pdg_status pdg_blk_create(pdg_ctx *ctx, int32_t H, int32_t W, const void *d_log_phi,
                          const void *d_log_unary, pdg_blk **out);
pdg_status pdg_blk_destroy(pdg_blk *b);

/* Advance the step counter s and draw every cut edge's dual from the
 * context's x (between sweeps; PDG_ESTATE otherwise). */
pdg_status pdg_blk_cut_duals(pdg_blk *b);
/* Network input rows from the current cut duals: d_in uint16 (BF16 bits)
 * [nb C][96]; optional d_target uint8 [nb C][64] (the block's current states,
 * training targets) and d_fields double [nb C][64] (f before rounding). */
pdg_status pdg_blk_inputs(pdg_blk *b, uint16_t *d_in, uint8_t *d_target, double *d_fields);
/* The Metropolis-Hastings move of every block and chain with the proposal
 * logits d_logits float [nb C][64]; accepted proposals are written to the
 * context's x.  Optional outputs per row: d_prop uint8 [nb C][64] the proposal,
 * d_acc uint8 [nb C] 1 if accepted, d_flag uint8 [nb C] 1 if a proposal
 * uniform lies within 1e-6 of its sigmoid(l) (evaluated in FP32) or log u
 * within 1e-9 of the log acceptance ratio (FP64): there the decision depends
 * on rounding. */
pdg_status pdg_blk_mh(pdg_blk *b, const float *d_logits, uint8_t *d_prop, uint8_t *d_acc,
                      uint8_t *d_flag);
/* Cut duals of the last pdg_blk_cut_duals: uint8 [m][C] in grid edge order
 * (0 on edges inside blocks). */
pdg_status pdg_blk_get_cut_duals(pdg_blk *b, uint8_t *d_theta);
/* Step counter, number of blocks, moves accepted and proposed so far. */
pdg_status pdg_blk_info(pdg_blk *b, int64_t *h_step, int64_t *h_blocks, int64_t *h_accepted,
                        int64_t *h_proposed);
pdg_status pdg_blk_set_step(pdg_blk *b, int64_t s);

/* Proposal network forward pass on `rows` input rows d_in (BF16 [rows][96]):
 * d_logits float [rows][64]; optional d_h1, d_h2 BF16 [rows][256], the two
 * hidden layers after ReLU (for the backward pass).  d_wbf / d_w32: the packed
 * parameters (BF16 weights, FP32 biases).  Enqueued on `stream`. */
pdg_status pdg_mlp_forward(const uint16_t *d_wbf, const float *d_w32, int64_t rows,
                           const uint16_t *d_in, float *d_logits, uint16_t *d_h1, uint16_t *d_h2,
                           void *stream);
/* Workspace bytes pdg_mlp_backward needs for `rows` rows. */
pdg_status pdg_mlp_backward_workspace(int64_t rows, int64_t *h_bytes);
/* Gradient of the mean over rows of the Bernoulli negative log-likelihood of
 * the targets d_target uint8 [rows][64] under the logits, into d_grad float
 * [PDG_MLP_PARAMS] (packed layout), and optionally the loss into *d_loss
 * (double, device).  The back-propagated matrices are rounded to BF16 for the
 * matrix cores; bias gradients are FP32 column sums of those BF16 values.
 * d_work: caller-owned workspace of pdg_mlp_backward_workspace bytes; on
 * return it holds the back-propagated BF16 matrices dL [rows][64] at byte 0,
 * dH2 [rows][256] at a(rows*128) and dH1 [rows][256] at a(rows*128) +
 * a(rows*512), a(k) = k rounded up to a multiple of 256 (for checks).
 * Enqueued on `stream`. */
pdg_status pdg_mlp_backward(const uint16_t *d_wbf, int64_t rows, const uint16_t *d_in,
                            const uint16_t *d_h1, const uint16_t *d_h2, const float *d_logits,
                            const uint8_t *d_target, float *d_grad, double *d_loss,
                            void *d_work, int64_t work_bytes, void *stream);
/* One Adam step (Kingma and Ba; bias-corrected, step >= 1) on the packed FP32
 * parameters d_w with gradient d_g and moments d_m, d_v (FP32, same layout);
 * refreshes the BF16 copy d_wbf.  Enqueued on `stream`. */
pdg_status pdg_mlp_adam(float *d_w, const float *d_g, float *d_m, float *d_v, int64_t step,
                        float lr, float beta1, float beta2, float eps, uint16_t *d_wbf,
                        void *stream);

/* The dense gather on the matrix cores (an experiment).  In a binary context
 * (q_max 2) with at most 16 chains, between the two phases of a sweep, writes
 * each listed node's field of state 1 given the current duals,
 * base_i(1) + sum_r 2 theta_r^c h_r over its incidence records, to d_out:
 * double [n][C].  method 0: vector FMAs (the hub kernels' arithmetic); method
 * 1: v_mfma_f64_16x16x4_f64 with the duals as a 16-chain x 4-record 0/1 matrix
 * and 2h in one column of 16 (a batched matrix-vector product: no operand is
 * shared between nodes).  Both FP64, results equal up to summation order.
 * d_nodes: int32 [n] node ids. */
pdg_status pdg_dense_fields(pdg_ctx *ctx, int64_t n, const int32_t *d_nodes, int32_t method,
                            double *d_out);

#ifdef __cplusplus
}
#endif

#endif /* PDG_BLOCK_H */
