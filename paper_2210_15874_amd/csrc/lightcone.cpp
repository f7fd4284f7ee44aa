// Lightcone tensor-network lowering (host side).
//
// The energy of a trajectory is sum_t w_t (1 - f_t <Z_u Z_v>_t) / 2, where
// <Z_u Z_v> is taken on the noiseless-structure state U(sigma)|0..0> of the
// Pauli-frame rewrite and f_t = +-1 is the final frame's sign on the term.
// For each term the planner keeps only the gates in the backward lightcone
// of {u, v} (the others cancel against their conjugates), builds the doubled
// network <0|U^dagger Z_u Z_v U|0> as tensors over binary variables (a
// diagonal gate reuses its qubits' current variables; any other gate opens
// new ones; the ket and bra chains of a qubit meet in one variable at the
// observable), orders the variables by min-fill with seeded random tie
// breaks, and lowers bucket elimination (Sec. III-A: contract the tensors
// that share the next variable, sum it out, return the result to the pool)
// into a list of steps.  Every trajectory shares the order and the steps;
// only the gate values (signs) differ, so the trajectory index is the batch
// dimension of the contraction kernel (kernels_tn.hip).
//
// Intermediates are placed by a first-fit allocator in two per-workgroup
// arenas: small ones in LDS while it has room, the others in global memory.
// A network whose intermediates all fit in LDS never touches global memory
// between its inputs and its result.
#include <algorithm>
#include <cmath>
#include <map>
#include <random>

#include "lightcone.h"

namespace stn {

namespace {

struct Tensor {
    int kind = TN_GATE;              // TnInputKind
    int gate = -1;                   // gate index (TN_GATE)
    int conj = 0;                    // bra side
    std::vector<int> vars;           // variable ids; local index bit k = vars[k]
    int arena = -1;                  // offset (TN_INTER)
    int lds = 0;                     // offset is in the LDS arena
};

bool diagonal_kind(uint32_t k) { return k == STN_G_RZ || k == STN_G_Z || k == STN_G_ZZ; }

// min-fill order of the interaction graph; ties broken by degree, then randomly.
// Stops (returning an empty order) as soon as the variable to eliminate has
// more than max_deg neighbours, i.e. a step of that rank would be needed;
// *deg_seen receives the largest degree met.
std::vector<int> minfill_order(int nv, const std::vector<std::vector<int>>& tensors, std::mt19937_64* rng,
                               int max_deg, int* deg_seen) {
    // adjacency as bit rows; fill and degree kept per variable and recomputed
    // only where an elimination changed a neighbourhood
    const size_t W = ((size_t)nv + 63) / 64;
    std::vector<uint64_t> A((size_t)nv * W, 0);
    auto row = [&](int v) { return A.data() + (size_t)v * W; };
    for (auto& t : tensors)
        for (int a : t)
            for (int b : t)
                if (a != b) row(a)[b >> 6] |= 1ull << (b & 63);
    std::vector<long> fill(nv, 0);
    std::vector<int> deg(nv, 0);
    // fill(v) = pairs of v's neighbours that are not adjacent: each neighbour a
    // counts the neighbours outside its own row, itself included, hence - deg
    auto recompute = [&](int v) {
        const uint64_t* r = row(v);
        int d = 0;
        for (size_t w = 0; w < W; ++w) d += __builtin_popcountll(r[w]);
        long f = 0;
        for (size_t w = 0; w < W; ++w)
            for (uint64_t m = r[w]; m; m &= m - 1) {
                const uint64_t* ra = row((int)(w * 64 + __builtin_ctzll(m)));
                for (size_t x = 0; x < W; ++x) f += __builtin_popcountll(r[x] & ~ra[x]);
            }
        deg[v] = d;
        fill[v] = (f - d) / 2;
    };
    for (int v = 0; v < nv; ++v) recompute(v);
    std::vector<char> done(nv, 0);
    std::vector<int> order;
    std::vector<uint64_t> nb(W), dirty(W);
    for (int it = 0; it < nv; ++it) {
        long best_fill = -1;
        int best_deg = 0;
        std::vector<int> cands;
        for (int v = 0; v < nv; ++v) {
            if (done[v]) continue;
            if (best_fill < 0 || fill[v] < best_fill || (fill[v] == best_fill && deg[v] < best_deg)) {
                best_fill = fill[v];
                best_deg = deg[v];
                cands.assign(1, v);
            } else if (fill[v] == best_fill && deg[v] == best_deg) {
                cands.push_back(v);
            }
        }
        int v = cands[0];
        if (rng && cands.size() > 1) v = cands[(*rng)() % cands.size()];
        *deg_seen = std::max(*deg_seen, best_deg);
        if (best_deg > max_deg) return {};
        done[v] = 1;
        order.push_back(v);
        // the neighbours of v become a clique; v leaves the graph
        std::copy(row(v), row(v) + W, nb.begin());
        std::fill(dirty.begin(), dirty.end(), 0ull);
        for (size_t w = 0; w < W; ++w)
            for (uint64_t m = nb[w]; m; m &= m - 1) {
                const int a = (int)(w * 64 + __builtin_ctzll(m));
                uint64_t* ra = row(a);
                for (size_t x = 0; x < W; ++x) ra[x] |= nb[x];
                ra[a >> 6] &= ~(1ull << (a & 63));
                ra[v >> 6] &= ~(1ull << (v & 63));
                for (size_t x = 0; x < W; ++x) dirty[x] |= ra[x];
            }
        std::fill(row(v), row(v) + W, 0ull);
        for (size_t w = 0; w < W; ++w) dirty[w] |= nb[w];
        for (size_t w = 0; w < W; ++w)
            for (uint64_t m = dirty[w]; m; m &= m - 1) {
                const int u = (int)(w * 64 + __builtin_ctzll(m));
                if (!done[u]) recompute(u);
            }
    }
    return order;
}

// bucket elimination along `order`; fills steps, returns (width, cost)
struct Lowered {
    std::vector<TnStepRec> steps;
    int width = 0;
    double cost = 0;         // sum over steps of 2^(vars in the step) * inputs
    int arena = 0;           // complex slots in global memory
    int lds_arena = 0;       // complex slots in LDS
    int result = -1;         // arena slot of the final scalar
    int result_lds = 0;
    double gbytes = 0;       // global-memory intermediates read and written
    std::vector<int> order;  // the elimination order lowered
};

// Intermediates of at most lds_tensor_max slots go to an LDS arena of
// lds_slots slots while it has room, all others to global memory.
struct TnArenaLimits {
    int lds_slots = 0;
    int lds_tensor_max = 0;
};

// First-fit placement of tensors in one arena of `cap` slots (cap < 0: unbounded).
struct FirstFit {
    std::map<int, int> used;  // offset -> size
    int cap = -1;
    int high = 0;             // slots used at most
    int alloc(int size) {     // -1 when it does not fit
        int off = 0;
        for (auto& kv : used) {
            if (kv.first - off >= size) break;
            off = std::max(off, kv.first + kv.second);
        }
        if (cap >= 0 && off + size > cap) return -1;
        used[off] = size;
        high = std::max(high, off + size);
        return off;
    }
    void release(int off) { used.erase(off); }
};

// Variables of every step of bucket elimination along `order` (the
// eliminated variable included), on variable lists without sliced variables.
std::vector<std::vector<int>> step_sets(const std::vector<std::vector<int>>& tv, const std::vector<int>& order) {
    std::vector<std::vector<int>> pool = tv, sets;
    std::vector<char> alive(pool.size(), 1);
    for (int v : order) {
        std::vector<int> out;
        bool any = false;
        for (size_t i = 0; i < pool.size(); ++i) {
            if (!alive[i] || std::find(pool[i].begin(), pool[i].end(), v) == pool[i].end()) continue;
            any = true;
            alive[i] = 0;
            for (int x : pool[i])
                if (x != v && std::find(out.begin(), out.end(), x) == out.end()) out.push_back(x);
        }
        if (!any) continue;
        std::vector<int> st = out;
        st.push_back(v);
        sets.push_back(st);
        pool.push_back(out);
        alive.push_back(1);
    }
    return sets;
}

// A step of bucket elimination before placement: input tensor ids, summed
// variables, output variables in storage order, output tensor id.
struct SymStep {
    std::vector<int> in;
    std::vector<int> sums;
    std::vector<int> out;
    int out_id = -1;
    bool dead = false;
};


// Bucket elimination along `order` (sliced variables skipped) in three
// phases: eliminate() does 1 and 2, place() does 3.
//  1. Each variable's bucket (the live tensors that hold it) becomes one step
//     whose output holds the bucket's other variables, in first-seen order
//     with the largest input first.
//  2. Merged-index steps: a step whose output's only reader sums one more
//     variable and adds nothing but small factors (all of whose variables
//     are in that output or summed there) is folded into its reader, which
//     then sums both variables over the same index space; the intermediate
//     is never written.  At most max_sums variables per step.
//  3. Intermediates are placed in step order (an output before its inputs
//     are released, so they never alias), small ones in LDS while it has
//     room, the others in global memory.
struct Symbolic {
    std::vector<Tensor> pool;      // base tensors, then one per step output
    std::vector<SymStep> steps;    // the last one multiplies the remaining scalars
    int result = -1;               // tensor id of the final scalar
};

// phases 1 and 2 (they do not depend on the placement)
Symbolic eliminate(const std::vector<Tensor>& base, const std::vector<int>& order, const std::vector<int>& sliced,
                   int max_sums) {
    auto is_sliced = [&](int x) { return std::find(sliced.begin(), sliced.end(), x) != sliced.end(); };
    // 1. symbolic elimination
    std::vector<Tensor> pool = base;
    std::vector<char> alive(pool.size(), 1);
    std::vector<SymStep> steps;
    for (int v : order) {
        if (is_sliced(v)) continue;
        std::vector<int> bucket;
        for (size_t i = 0; i < pool.size(); ++i)
            if (alive[i] && std::find(pool[i].vars.begin(), pool[i].vars.end(), v) != pool[i].vars.end())
                bucket.push_back((int)i);
        if (bucket.empty()) continue;
        std::stable_sort(bucket.begin(), bucket.end(),
                         [&](int a, int b) { return pool[a].vars.size() > pool[b].vars.size(); });
        SymStep st;
        st.in = bucket;
        st.sums = {v};
        for (int i : bucket)
            for (int x : pool[i].vars)
                if (x != v && !is_sliced(x) && std::find(st.out.begin(), st.out.end(), x) == st.out.end())
                    st.out.push_back(x);
        for (int i : bucket) alive[i] = 0;
        Tensor t;
        t.kind = TN_INTER;
        t.vars = st.out;
        st.out_id = (int)pool.size();
        pool.push_back(t);
        alive.push_back(1);
        steps.push_back(st);
    }
    SymStep fin;   // remaining scalars (no variables but sliced ones) multiply into the result
    for (size_t i = 0; i < pool.size(); ++i)
        if (alive[i]) {
            for (int x : pool[i].vars)
                if (!is_sliced(x)) fail(STN_E_INVALID, "tensor left with open indices");
            fin.in.push_back((int)i);
        }
    Tensor res;
    res.kind = TN_INTER;
    fin.out_id = (int)pool.size();
    pool.push_back(res);
    steps.push_back(fin);
    const int result = fin.out_id;
    // 2. merged-index steps
    std::vector<int> reader(pool.size(), -1);
    for (size_t k = 0; k < steps.size(); ++k)
        for (int i : steps[k].in) reader[i] = (int)k;
    for (size_t k = 0; k + 1 < steps.size(); ++k) {
        SymStep& s = steps[k];
        const int c = reader[s.out_id];
        if (c < 0 || steps[c].sums.empty() || (int)(s.sums.size() + steps[c].sums.size()) > max_sums) continue;
        SymStep& r = steps[c];
        bool small_only = true;
        for (int i : r.in) {
            if (i == s.out_id) continue;
            for (int x : pool[i].vars)
                if (!is_sliced(x) && std::find(s.out.begin(), s.out.end(), x) == s.out.end() &&
                    std::find(r.sums.begin(), r.sums.end(), x) == r.sums.end())
                    small_only = false;
            if (pool[i].vars.size() > 2) small_only = false;
        }
        if (!small_only) continue;
        std::vector<int> in = s.in;
        for (int i : r.in)
            if (i != s.out_id) in.push_back(i);
        std::vector<int> sums = s.sums;
        sums.insert(sums.end(), r.sums.begin(), r.sums.end());
        r.in = in;
        r.sums = sums;
        for (int i : r.in) reader[i] = c;
        s.dead = true;
    }
    Symbolic out;
    out.pool = std::move(pool);
    out.steps = std::move(steps);
    out.result = result;
    return out;
}

// phase 3: placement of the intermediates (the symbolic pool is only read)
Lowered place(const Symbolic& sym, const std::vector<int>& order, const std::vector<int>& sliced,
              TnArenaLimits lim) {
    Lowered L;
    auto slice_bit = [&](int x) {
        const auto it = std::find(sliced.begin(), sliced.end(), x);
        return it == sliced.end() ? -1 : (int)(it - sliced.begin());
    };
    const std::vector<Tensor>& pool = sym.pool;
    std::vector<int> arena(pool.size(), -1);
    std::vector<char> in_lds(pool.size(), 0);
    FirstFit gmem, lds;
    lds.cap = lim.lds_slots;
    auto alloc = [&](int id, int size) {
        if (size <= lim.lds_tensor_max) {
            const int off = lds.alloc(size);
            if (off >= 0) {
                in_lds[id] = 1;
                arena[id] = off;
                return;
            }
        }
        arena[id] = gmem.alloc(size);
    };
    auto release = [&](int id) { (in_lds[id] ? lds : gmem).release(arena[id]); };
    for (auto& st : sym.steps) {
        if (st.dead) continue;
        TnStepRec rec;
        rec.elim = st.sums.empty() ? -1 : st.sums[0];
        rec.nsum = (int)st.sums.size();
        rec.out_vars = st.out;
        const int full = (int)st.out.size() + rec.nsum;
        L.width = std::max(L.width, full);
        L.cost += std::ldexp(1.0, full) * st.in.size();
        for (int i : st.in) {
            TnInputRec in;
            in.kind = pool[i].kind;
            in.gate = pool[i].gate;
            in.conj = pool[i].conj;
            in.arena = arena[i];
            in.lds = in_lds[i];
            // position of each of the input's variables in the step's index space
            // (output variables at bits 0..|out|-1, the summed ones from |out|;
            // a sliced variable: its bit of the slice index)
            for (int x : pool[i].vars) {
                const int sb = slice_bit(x);
                if (sb >= 0) {
                    in.pos.push_back(-1 - sb);
                    continue;
                }
                const auto it = std::find(st.out.begin(), st.out.end(), x);
                if (it != st.out.end()) {
                    in.pos.push_back((int)(it - st.out.begin()));
                } else {
                    const auto is = std::find(st.sums.begin(), st.sums.end(), x);
                    if (is == st.sums.end()) fail(STN_E_INVALID, "lightcone lowering: input variable not in its step");
                    in.pos.push_back((int)st.out.size() + (int)(is - st.sums.begin()));
                }
            }
            rec.inputs.push_back(std::move(in));
        }
        // the output is placed while the inputs are still held: no aliasing
        alloc(st.out_id, 1 << st.out.size());
        for (int i : st.in)
            if (pool[i].kind == TN_INTER) {
                if (!in_lds[i]) L.gbytes += std::ldexp(1.0, (int)pool[i].vars.size());
                release(i);
            }
        if (!in_lds[st.out_id]) L.gbytes += std::ldexp(1.0, (int)st.out.size());
        rec.out_arena = arena[st.out_id];
        rec.out_lds = in_lds[st.out_id];
        L.steps.push_back(std::move(rec));
    }
    L.result = arena[sym.result];
    L.result_lds = in_lds[sym.result];
    L.arena = gmem.high;
    L.lds_arena = lds.high;
    L.order = order;
    return L;
}

// Lowers `order` for an LDS arena of lds_slots slots with tensor caps of the
// whole arena, a quarter and a sixteenth of it, and keeps the lowering that
// moves the fewest bytes through global memory (a large tensor kept in LDS
// can push several smaller ones out).
Lowered lower_best_placement(const Symbolic& sym, const std::vector<int>& order, const std::vector<int>& sliced,
                             int lds_slots) {
    TnArenaLimits lim;
    lim.lds_slots = lds_slots;
    lim.lds_tensor_max = lds_slots;
    Lowered best = place(sym, order, sliced, lim);
    for (int cap = lds_slots / 4; cap >= 64 && cap >= lds_slots / 16; cap /= 4) {
        lim.lds_tensor_max = cap;
        Lowered L = place(sym, order, sliced, lim);
        if (L.gbytes < best.gbytes) best = std::move(L);
    }
    return best;
}

// merged-index steps (two summed variables) in complex64 plans only
int max_sums(const stn_plan* p) { return p->opts.precision == 128 ? 1 : 2; }

void take(TnNetwork& net, Lowered&& L) {
    net.steps = std::move(L.steps);
    net.width = L.width;
    net.cost = L.cost;
    net.arena = L.arena;
    net.lds_arena = L.lds_arena;
    net.result = L.result;
    net.result_lds = L.result_lds;
}

// The caller's order for one term's network: validated as a permutation of
// the variables, checked against max_rank, then lowered unsliced.
std::vector<TnNetwork> lower_caller_order(const stn_plan* p, uint32_t term, const std::vector<Tensor>& ts, int nv,
                                          int max_rank, TnNetwork net, const std::vector<int>& lds_slots) {
    std::vector<uint32_t> offsets(1, 0), vars;
    std::vector<std::vector<int>> tv;
    for (auto& t : ts) {
        for (int x : t.vars) vars.push_back((uint32_t)x);
        offsets.push_back((uint32_t)vars.size());
        tv.push_back(t.vars);
    }
    stn_term_network desc;
    desc.term = term;
    desc.u = net.u;
    desc.v = net.v;
    desc.n_vars = (uint32_t)nv;
    desc.n_tensors = (uint32_t)ts.size();
    desc.tensor_offsets = offsets.data();
    desc.tensor_vars = vars.data();
    std::vector<uint32_t> got((size_t)nv, 0);
    if (p->opts.lc_order_fn(&desc, got.data(), p->opts.lc_order_ctx) != 0)
        fail(STN_E_INVALID, "contraction order rejected by the caller for term " + std::to_string(term));
    std::vector<char> seen((size_t)nv, 0);
    std::vector<int> order;
    for (uint32_t x : got) {
        if (x >= (uint32_t)nv || seen[x])
            fail(STN_E_INVALID, "contraction order of term " + std::to_string(term) + " is not a permutation of its " +
                                    std::to_string(nv) + " variables");
        seen[x] = 1;
        order.push_back((int)x);
    }
    int widest = 0;
    for (auto& st : step_sets(tv, order)) widest = std::max(widest, (int)st.size());
    if (widest > max_rank + 1) {
        net.width = widest;
        net.cost = HUGE_VAL;
        return std::vector<TnNetwork>(lds_slots.size(), net);
    }
    std::vector<TnNetwork> out;
    const Symbolic sym = eliminate(ts, order, {}, max_sums(p));
    for (int slots : lds_slots) {
        TnNetwork n2 = net;
        take(n2, lower_best_placement(sym, order, {}, slots));
        out.push_back(std::move(n2));
    }
    return out;
}

}  // namespace

// Network of one term: lightcone gates on the ket, the observable, the
// conjugate gates on the bra, |0> at both ends of every chain.
std::vector<TnNetwork> build_term(const stn_plan* p, uint32_t term, uint32_t u, uint32_t v, uint32_t restarts,
                                  uint64_t seed, int max_rank, int slice_bits, const std::vector<int>& lds_slots) {
    const uint32_t n = p->n;
    // backward lightcone of {u, v}
    std::vector<char> in_cone(p->gates.size(), 0);
    uint64_t S = (1ull << u) | (1ull << v);
    for (size_t gi = p->gates.size(); gi-- > 0;) {
        const GateRec& g = p->gates[gi];
        const uint64_t qm = (1ull << g.q0) | (g.nq == 2 ? (1ull << g.q1) : 0);
        if (S & qm) {
            in_cone[gi] = 1;
            S |= qm;
        }
    }
    // ket chain
    int nv = 0;
    std::vector<int> cur(n, -1), first(n, -1);
    std::vector<Tensor> ts;
    auto var_of = [&](uint32_t q) {
        if (cur[q] < 0) {
            cur[q] = first[q] = nv++;
        }
        return cur[q];
    };
    std::vector<int> cone_gates;
    for (size_t gi = 0; gi < p->gates.size(); ++gi)
        if (in_cone[gi]) cone_gates.push_back((int)gi);
    auto add_gate = [&](int gi, int conj, std::vector<int>& curv, std::vector<int>& firstv) {
        const GateRec& g = p->gates[gi];
        auto v_of = [&](uint32_t q) {
            if (curv[q] < 0) curv[q] = firstv[q] = nv++;
            return curv[q];
        };
        Tensor t;
        t.kind = TN_GATE;
        t.gate = gi;
        t.conj = conj;
        if (diagonal_kind(g.kind)) {
            t.vars.push_back(v_of(g.q0));
            if (g.nq == 2) t.vars.push_back(v_of(g.q1));
        } else if (g.nq == 1) {
            // local index bit 0 = input variable, bit 1 = output variable
            const int in = v_of(g.q0);
            const int out = nv++;
            curv[g.q0] = out;
            t.vars = {in, out};
        } else {
            const int in0 = v_of(g.q0), in1 = v_of(g.q1);
            const int o0 = nv++, o1 = nv++;
            curv[g.q0] = o0;
            curv[g.q1] = o1;
            t.vars = {in0, in1, o0, o1};
        }
        ts.push_back(t);
    };
    (void)var_of;
    for (int gi : cone_gates) add_gate(gi, 0, cur, first);
    // observable on the final ket variables, shared with the bra
    {
        std::vector<int> dummy;
        Tensor o;
        o.kind = TN_OBS;
        if (cur[u] < 0) cur[u] = first[u] = nv++;
        if (cur[v] < 0) cur[v] = first[v] = nv++;
        o.vars = {cur[u], cur[v]};
        ts.push_back(o);
    }
    // bra chain, walked backward from the shared final variables
    std::vector<int> bcur = cur, bfirst(n, -1);
    for (size_t k = cone_gates.size(); k-- > 0;) {
        const GateRec& g = p->gates[cone_gates[k]];
        Tensor t;
        t.kind = TN_GATE;
        t.gate = cone_gates[k];
        t.conj = 1;
        if (diagonal_kind(g.kind)) {
            t.vars.push_back(bcur[g.q0]);
            if (g.nq == 2) t.vars.push_back(bcur[g.q1]);
        } else if (g.nq == 1) {
            const int out = bcur[g.q0];  // the gate's output side is later in time
            const int in = nv++;
            bcur[g.q0] = in;
            t.vars = {in, out};
        } else {
            const int o0 = bcur[g.q0], o1 = bcur[g.q1];
            const int i0 = nv++, i1 = nv++;
            bcur[g.q0] = i0;
            bcur[g.q1] = i1;
            t.vars = {i0, i1, o0, o1};
        }
        ts.push_back(t);
    }
    // |0> at the start of both chains of every qubit that appears
    for (uint32_t q = 0; q < n; ++q) {
        if (first[q] >= 0) {
            Tensor z;
            z.kind = TN_ZERO;
            z.vars = {first[q]};
            ts.push_back(z);
        }
        if (cur[q] >= 0 && bcur[q] >= 0 && bcur[q] != first[q]) {
            Tensor z;
            z.kind = TN_ZERO;
            z.vars = {bcur[q]};
            ts.push_back(z);
        } else if (cur[q] >= 0 && bcur[q] == first[q] && first[q] >= 0) {
            // qubit with no non-diagonal gate: ket and bra start share one variable
        }
    }
    TnNetwork net;
    net.u = u;
    net.v = v;
    net.n_vars = nv;
    if (p->opts.lc_order_fn) return lower_caller_order(p, term, ts, nv, max_rank, net, lds_slots);
    struct Scored {
        std::vector<int> order;
        int width = 0;
        double cost = 0;
    } best;
    bool have = false;
    std::vector<int> sliced;   // slice index bit k fixes variable sliced[k]
    int deg_lb = 0;
    for (;;) {
        // interaction graph without the sliced variables
        std::vector<std::vector<int>> tv;
        for (auto& t : ts) {
            std::vector<int> r;
            for (int x : t.vars)
                if (std::find(sliced.begin(), sliced.end(), x) == sliced.end()) r.push_back(x);
            tv.push_back(r);
        }
        std::mt19937_64 rng(seed ^ (0x9E3779B97F4A7C15ull * (u * 131 + v)));
        deg_lb = 0;
        for (uint32_t r = 0; r <= restarts; ++r) {
            int deg = 0;
            const std::vector<int> order = minfill_order(nv, tv, r == 0 ? nullptr : &rng, max_rank, &deg);
            if (order.empty() && nv > 0) {   // this order needs a step above max_rank
                deg_lb = deg_lb ? std::min(deg_lb, deg) : deg;
                continue;
            }
            // width and work of the plain elimination (no merging or placement)
            const Symbolic sym = eliminate(ts, order, sliced, 1);
            Scored sc;
            for (auto& st : sym.steps) {
                const int full = (int)(st.out.size() + st.sums.size());
                sc.width = std::max(sc.width, full);
                sc.cost += std::ldexp(1.0, full) * st.in.size();
            }
            if (!have || sc.width < best.width || (sc.width == best.width && sc.cost < best.cost)) {
                sc.order = order;
                best = std::move(sc);
                have = true;
            }
        }
        if (have || (int)sliced.size() >= slice_bits) break;
        // slice the variable that sits in the most (and widest) steps above
        // max_rank of an unbounded-rank min-fill order, then try again
        int deg = 0;
        const std::vector<int> order = minfill_order(nv, tv, nullptr, nv, &deg);
        std::vector<double> score(nv, 0.0);
        for (auto& st : step_sets(tv, order))
            if ((int)st.size() > max_rank + 1)
                for (int x : st) score[x] += std::ldexp(1.0, (int)st.size() - max_rank - 1);
        int pick = -1;
        for (int x = 0; x < nv; ++x)
            if (score[x] > 0 && (pick < 0 || score[x] > score[pick])) pick = x;
        if (pick < 0) break;
        sliced.push_back(pick);
    }
    if (!have) {   // no order within max_rank: width is at least deg_lb + 1
        net.width = deg_lb + 1;
        net.cost = HUGE_VAL;
        return std::vector<TnNetwork>(lds_slots.size(), net);
    }
    net.slice_bits = (int)sliced.size();
    std::vector<TnNetwork> out;
    const Symbolic sym = eliminate(ts, best.order, sliced, max_sums(p));
    for (int slots : lds_slots) {
        TnNetwork n2 = net;
        take(n2, lower_best_placement(sym, best.order, sliced, slots));
        n2.cost = std::ldexp(n2.cost, n2.slice_bits);
        out.push_back(std::move(n2));
    }
    return out;
}

}  // namespace stn
