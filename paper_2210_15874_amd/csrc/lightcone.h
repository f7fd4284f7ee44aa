// Lightcone tensor-network lowering: host records shared by the planner
// (lightcone.cpp) and the contraction kernel (kernels_tn.hip).
#pragma once

#include "stn_internal.h"

namespace stn {

enum TnInputKind : int32_t {
    TN_GATE = 0,     // a circuit gate's tensor (values from the gate and the trajectory's sign)
    TN_OBS = 1,      // Z_u Z_v on the two shared final variables
    TN_ZERO = 2,     // |0> at the start of a chain
    TN_INTER = 3     // an intermediate result in the arena
};

struct TnInputRec {
    int kind = TN_GATE;
    int gate = -1;
    int conj = 0;
    int arena = -1;
    int lds = 0;                   // TN_INTER: the tensor lives in the workgroup's LDS arena
    // local index bit k of the input = bit pos[k] of the step's index, or,
    // where pos[k] < 0, bit -1 - pos[k] of the slice index
    std::vector<int> pos;
};

struct TnStepRec {
    int elim = -1;                 // first summed variable (-1: the final product of scalars)
    int nsum = 0;                  // summed variables (step index bits out_vars.size() ..); more than one
                                   // when consecutive eliminations are merged into one step
    std::vector<int> out_vars;
    std::vector<TnInputRec> inputs;
    int out_arena = -1;
    int out_lds = 0;               // the output goes to the LDS arena
};

struct TnNetwork {
    uint32_t u = 0, v = 0;
    int n_vars = 0;
    int width = 0;                 // largest step index space (output rank + 1), per slice
    int slice_bits = 0;            // variables fixed by the slice index (2^slice_bits slices, summed)
    double cost = 0;               // sum over steps of 2^width(step) * inputs, times the slices
    int arena = 0;                 // complex slots of intermediates in global memory
    int lds_arena = 0;             // complex slots of intermediates in LDS
    int result = -1;               // arena slot of the final scalar
    int result_lds = 0;            // ... in the LDS arena
    std::vector<TnStepRec> steps;
};

// Networks whose elimination order would need a step of rank above max_rank
// are sliced (Sec. III-C: variables fixed to each of their values, the
// results summed) by up to slice_bits variables; those still too wide come
// back without steps, width = a lower bound, cost = infinity.  With a
// caller-supplied order (opts.lc_order_fn) that order is lowered instead of
// min-fill, unsliced; a network it leaves too wide comes back the same way.
// The order found is lowered once per LDS budget in lds_slots (one network
// each, same order): intermediates are placed in an LDS arena of that many
// slots while it has room (first fit), all others in global memory.
std::vector<TnNetwork> build_term(const stn_plan* p, uint32_t term, uint32_t u, uint32_t v, uint32_t restarts,
                                  uint64_t seed, int max_rank, int slice_bits, const std::vector<int>& lds_slots);

}  // namespace stn
