// What other parts of the library (the learned block proposal) may see of a
// sampler context, and how they report errors through pdg_last_error.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "pdg.h"

namespace pdg {

struct CtxView {
    int device;
    hipStream_t stream;
    uint8_t *d_x;        // [n][C] chain states
    const uint8_t *d_q;  // [n] states per node
    int64_t n;
    int32_t C, QM, precision;
    uint64_t seed;
    int phase;  // 0 between sweeps, 1 between the dual and the primal phase
    // incidence records (each node's segment [off, off + cnt) of the pool):
    // h [pool][RP] in the node's orientation, dual mask words [pool][ZW]
    const double *rec_p;
    const uint32_t *rec_z;
    const uint32_t *inc_off, *inc_cnt;
    const double *base;  // [n][QM] log unaries plus the records' theta-free fields
    int32_t RP;
    int64_t ZW;
};

// Fills *v and makes the context's device current; a failure (a broken
// context, a HIP error) is reported on ctx and returned.
pdg_status ctx_view(pdg_ctx *ctx, CtxView *v);
// Records msg as ctx's last error (ctx == nullptr: the global one); returns code.
pdg_status report(pdg_ctx *ctx, pdg_status code, const std::string &msg);

}  // namespace pdg
