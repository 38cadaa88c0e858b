/*
 * pdg_rates.h -- instruction-rate measurement behind the sweep's VALU roofline
 * (built into libpdg.so).  Not part of the sampler: it times, on the current
 * device, three loops that every lane of a full grid runs with independent
 * dependency chains, and reports lane-operations per second:
 *   [0] 32-bit integer adds (v_add_u32), a full-rate reference op;
 *   [1] 32 x 32 -> 64-bit multiply-adds (v_mad_u64_u32), the product of a
 *       Philox round;
 *   [2] complete Philox4x32-10 calls (the generator of the dual and primal
 *       phases), counted as calls.
 * The dual's algorithmic cost per draw (one fifth of a call plus three
 * compares) is priced in full-rate slots from these numbers.
 */
#ifndef PDG_RATES_H
#define PDG_RATES_H

#include <stdint.h>

#include "pdg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Runs each loop `iters` iterations per lane (1 <= iters <= 2^24) on `device`
 * after one warm-up launch and writes the three rates (per second, summed over
 * all lanes) to h_out[3] (host).  Allocates and frees a small device buffer;
 * synchronizes the device.  PDG_EINVAL on bad arguments, PDG_EHIP on a HIP
 * error. */
pdg_status pdg_valu_rates(int32_t device, int64_t iters, double *h_out);

#ifdef __cplusplus
}
#endif

#endif /* PDG_RATES_H */
