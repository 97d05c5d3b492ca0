// Internal interface between the batch host code and the column kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tplbm.h"
#include "lbm_common.hpp"

namespace tplbm {

struct ColumnDesc {
    int32_t height;   // nodes, both wall nodes included
    int32_t form;     // gravity form 1, 2 or 3
    int64_t offset;   // first node in the concatenated arrays
    double g;         // gravity magnitude, positive downward
    double rho_v;     // form 3: the subtracted vapour density
};

struct ColumnResult {
    int64_t steps;    // level at which the run stopped
    int32_t status;   // 0 converged, 1 diverged, 2 step budget reached
    int32_t pad;
    double mass;      // sum of rho at that level
    double max_u;     // max |u| at that level
};

struct BatchArgs {
    const ColumnDesc *cols;
    int ncols;
    const int *order;       // processing order (indices into cols)
    const double *rho0, *T0;
    double *rho_out, *T_out;
    // populations of a previous run's end level (f0, f+, f- planes of
    // `nodes` values each) to continue from instead of rest populations of
    // rho0; NULL starts at rest.  The end level's populations go to f_out.
    // f_in may equal f_out, and T0 may equal T_out: a column's nodes are read
    // only by the block that runs it, before that block writes them.  f_out
    // NULL: the end populations are not kept.
    const double *f_in;
    double *f_out;
    int64_t nodes;
    ColumnResult *results;
    unsigned *queue;        // next position in `order`; zero before a launch
    double tol;
    int check_every;
    int64_t max_steps;
};

struct BatchShape {
    int threads, nodes_per_thread;
};

extern const BatchShape kBatchShapes[];
extern const int kNumBatchShapes;
hipError_t d1q3_batch_launch(int shape, const BatchArgs &a, const Phys &c, int grid, hipStream_t s);
hipError_t d1q3_batch_occupancy(int shape, int *blocks_per_cu);

// Host helpers shared by the batch entry points (batch_host.cpp).
// Validate batch parameters and columns; *total receives the node count.
// On failure the message goes to the calling thread's context-free error.
int batch_validate(const tplbm_batch_params *p, int32_t ncols, const tplbm_column *cols, int64_t *total);
// Record a context-free failure (tplbm_batch_last_error(NULL)) and return code.
int batch_fail(int code, const char *fmt, ...);
Phys batch_phys(const tplbm_batch_params &p);
// Persistent grid of a shape: resident workgroups on the current device, at most ncols.
int batch_grid(int shape, int ncols);

}  // namespace tplbm
