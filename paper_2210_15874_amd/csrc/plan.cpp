// Host planner: validates a circuit + noise model, builds the noise-site
// table (selection probabilities, integer thresholds, inserted operators),
// the Pauli-frame tables and one of the lowerings declared in stn.h.
//
// Compiled with -ffp-contract=off: the thresholds must be bit-identical to
// any other implementation that follows the stated evaluation order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <sstream>

#include "stn_internal.h"

namespace stn {

namespace {

const cd I1(0, 1);

std::vector<cd> pauli_matrix(int a) {
    switch (a) {
        case 0: return {1, 0, 0, 1};
        case 1: return {0, 1, 1, 0};
        case 2: return {0, -I1, I1, 0};
        default: return {1, 0, 0, -1};
    }
}

// kron for little-endian local indices: result acts with `lo` on local bit 0
std::vector<cd> kron_le(const std::vector<cd>& hi, const std::vector<cd>& lo) {
    std::vector<cd> r(16);
    for (int oh = 0; oh < 2; ++oh)
        for (int ol = 0; ol < 2; ++ol)
            for (int ih = 0; ih < 2; ++ih)
                for (int il = 0; il < 2; ++il)
                    r[(ol + 2 * oh) * 4 + (il + 2 * ih)] = hi[oh * 2 + ih] * lo[ol * 2 + il];
    return r;
}

std::string where_gate(uint32_t g) { return "gate " + std::to_string(g); }
std::string where_site(uint32_t s) { return "channel " + std::to_string(s); }

void gate_record(GateRec& r, const stn_gate& g, uint32_t n, uint32_t gi) {
    r.kind = g.kind;
    r.q0 = g.q0;
    r.q1 = g.q1;
    r.theta = g.theta;
    const bool two = g.kind == STN_G_ZZ || g.kind == STN_G_CX || g.kind == STN_G_U2;
    r.nq = two ? 2 : 1;
    if (g.kind > STN_G_U2) fail(STN_E_INVALID, where_gate(gi) + ": unknown gate kind");
    if (g.q0 >= n || (two && g.q1 >= n)) fail(STN_E_INVALID, where_gate(gi) + ": qubit out of range");
    if (two && g.q0 == g.q1) fail(STN_E_INVALID, where_gate(gi) + ": repeated qubit");
    if (!std::isfinite(g.theta)) fail(STN_E_INVALID, where_gate(gi) + ": non-finite angle");
    const double c = std::cos(g.theta / 2), s = std::sin(g.theta / 2);
    const uint64_t b0 = 1ull << g.q0, b1 = two ? (1ull << g.q1) : 0;
    switch (g.kind) {
        case STN_G_H: {
            const double h = 1.0 / std::sqrt(2.0);
            r.m = {h, h, h, -h};
            break;
        }
        case STN_G_X: r.m = pauli_matrix(1); break;
        case STN_G_Y: r.m = pauli_matrix(2); break;
        case STN_G_Z: r.m = pauli_matrix(3); break;
        case STN_G_RX:
            r.m = {c, -I1 * s, -I1 * s, c};
            r.rotation = true; r.gx = b0;
            break;
        case STN_G_RY:
            r.m = {c, -s, s, c};
            r.rotation = true; r.gx = b0; r.gz = b0;
            break;
        case STN_G_RZ:
            r.m = {std::exp(-I1 * (g.theta / 2)), 0, 0, std::exp(I1 * (g.theta / 2))};
            r.rotation = true; r.gz = b0;
            break;
        case STN_G_ZZ: {
            const cd e = std::exp(-I1 * g.theta);
            r.m.assign(16, 0);
            r.m[0] = 1; r.m[5] = e; r.m[10] = e; r.m[15] = 1;
            r.rotation = true; r.gz = b0 | b1;
            break;
        }
        case STN_G_CX: {
            r.m.assign(16, 0);
            for (int cb = 0; cb < 2; ++cb)
                for (int t = 0; t < 2; ++t) r.m[(cb | ((t ^ cb) << 1)) * 4 + (cb | (t << 1))] = 1;
            break;
        }
        case STN_G_U1:
        case STN_G_U2: {
            if (!g.mat) fail(STN_E_INVALID, where_gate(gi) + ": explicit gate without matrix");
            const int d = g.kind == STN_G_U1 ? 2 : 4;
            r.m.resize(d * d);
            for (int i = 0; i < d * d; ++i) {
                r.m[i] = cd(g.mat[2 * i], g.mat[2 * i + 1]);
                if (!std::isfinite(g.mat[2 * i]) || !std::isfinite(g.mat[2 * i + 1]))
                    fail(STN_E_INVALID, where_gate(gi) + ": non-finite matrix entry");
            }
            break;
        }
    }
}

// Selection probabilities in the closed forms of the named channels; the
// evaluation order is part of the bit-exactness contract of the thresholds.
std::vector<double> selection_probs(const stn_channel& ch, const std::vector<std::vector<cd>>& ops, int d) {
    const double lam = ch.param;
    switch (ch.kind) {
        case STN_CH_BITFLIP: return {lam, 1.0 - lam};
        case STN_CH_DEPOL1: {
            const double qp = lam / 4.0;
            return {1.0 - 3.0 * qp, qp, qp, qp};
        }
        case STN_CH_DEPOL2: {
            const double qp = lam / 16.0;
            std::vector<double> q(16, qp);
            q[0] = 1.0 - 15.0 * qp;
            return q;
        }
        case STN_CH_AMPDAMP: return {1.0 - lam / 2.0, lam / 2.0};
        default: {
            std::vector<double> q;
            for (auto& K : ops) {
                double s = 0.0;
                for (auto& v : K) s = s + (v.real() * v.real() + v.imag() * v.imag());
                q.push_back(s / d);
            }
            return q;
        }
    }
}

std::vector<uint64_t> thresholds(const std::vector<double>& q) {
    std::vector<uint64_t> T(q.size());
    double c = 0.0;
    for (size_t j = 0; j < q.size(); ++j) {
        c = c + q[j];
        if (j + 1 == q.size()) {
            T[j] = 1ull << 32;
        } else {
            const double f = std::floor(c * 4294967296.0);
            T[j] = f >= 4294967296.0 ? (1ull << 32) : (f <= 0 ? 0 : (uint64_t)f);
        }
    }
    return T;
}

// Is op proportional (|c| = 1) to a Pauli string on the channel's qubits?
bool as_pauli(const std::vector<cd>& op, int nq, uint32_t q0, uint32_t q1, uint64_t& xm, uint64_t& zm) {
    const int d = 1 << nq;
    for (int code = 0; code < (1 << (2 * nq)); ++code) {
        const int a0 = code & 3, a1 = (code >> 2) & 3;
        std::vector<cd> P = nq == 1 ? pauli_matrix(a0) : kron_le(pauli_matrix(a1), pauli_matrix(a0));
        cd c = 0;
        for (int i = 0; i < d * d; ++i) c += std::conj(P[i]) * op[i];
        c /= double(d);
        if (std::abs(std::abs(c) - 1.0) > 1e-12) continue;
        double err = 0;
        for (int i = 0; i < d * d; ++i) err = std::max(err, std::abs(op[i] - c * P[i]));
        if (err > 1e-12) continue;
        xm = zm = 0;
        auto put = [&](int a, uint32_t q) {
            if (a == 1 || a == 2) xm |= 1ull << q;
            if (a == 2 || a == 3) zm |= 1ull << q;
        };
        put(a0, q0);
        if (nq == 2) put(a1, q1);
        return true;
    }
    return false;
}

void site_record(SiteRec& r, const stn_channel& ch, uint32_t n, uint32_t n_gates, uint32_t si) {
    r.gate = ch.after_gate;
    r.nq = ch.n_qubits;
    r.q0 = ch.q0;
    r.q1 = ch.q1;
    if (ch.after_gate >= n_gates) fail(STN_E_INVALID, where_site(si) + ": after_gate out of range");
    if (ch.kind > STN_CH_KRAUS) fail(STN_E_INVALID, where_site(si) + ": unknown channel kind");
    const bool named2 = ch.kind == STN_CH_DEPOL2;
    if (named2 && ch.n_qubits != 2) fail(STN_E_INVALID, where_site(si) + ": depol2 needs 2 qubits");
    if ((ch.kind == STN_CH_BITFLIP || ch.kind == STN_CH_DEPOL1 || ch.kind == STN_CH_AMPDAMP) && ch.n_qubits != 1)
        fail(STN_E_INVALID, where_site(si) + ": one-qubit channel with n_qubits != 1");
    if (ch.n_qubits < 1 || ch.n_qubits > 2) fail(STN_E_INVALID, where_site(si) + ": n_qubits must be 1 or 2");
    if (ch.q0 >= n || (ch.n_qubits == 2 && (ch.q1 >= n || ch.q1 == ch.q0)))
        fail(STN_E_INVALID, where_site(si) + ": qubit out of range or repeated");
    if (ch.kind != STN_CH_KRAUS && !(ch.param >= 0.0 && ch.param <= 1.0))
        fail(STN_E_INVALID, where_site(si) + ": parameter outside [0, 1]");
    const int d = 1 << ch.n_qubits;
    std::vector<std::vector<cd>> K;
    std::vector<std::pair<int, int>> labels;  // Pauli labels (a0, a1) of named Pauli channels
    const double lam = ch.param;
    switch (ch.kind) {
        case STN_CH_BITFLIP:
            K = {pauli_matrix(1), pauli_matrix(0)};
            for (auto& v : K[0]) v *= std::sqrt(lam);
            for (auto& v : K[1]) v *= std::sqrt(1.0 - lam);
            labels = {{1, 0}, {0, 0}};
            break;
        case STN_CH_DEPOL1:
            for (int a = 0; a < 4; ++a) {
                auto P = pauli_matrix(a);
                const double w = a == 0 ? 1.0 - 3.0 * lam / 4.0 : lam / 4.0;
                for (auto& v : P) v *= std::sqrt(w);
                K.push_back(P);
                labels.push_back({a, 0});
            }
            break;
        case STN_CH_DEPOL2:
            for (int j = 0; j < 16; ++j) {
                auto P = kron_le(pauli_matrix(j % 4), pauli_matrix(j / 4));
                const double w = j == 0 ? 1.0 - 15.0 * lam / 16.0 : lam / 16.0;
                for (auto& v : P) v *= std::sqrt(w);
                K.push_back(P);
                labels.push_back({j / 4, j % 4});
            }
            break;
        case STN_CH_AMPDAMP:
            K = {{1, 0, 0, std::sqrt(1.0 - lam)}, {0, std::sqrt(lam), 0, 0}};
            break;
        case STN_CH_KRAUS:
            if (ch.n_kraus < 1 || ch.n_kraus > 16 || !ch.kraus)
                fail(STN_E_INVALID, where_site(si) + ": explicit channel needs 1..16 Kraus operators");
            for (uint32_t j = 0; j < ch.n_kraus; ++j) {
                std::vector<cd> m(d * d);
                for (int i = 0; i < d * d; ++i) {
                    m[i] = cd(ch.kraus[(j * d * d + i) * 2], ch.kraus[(j * d * d + i) * 2 + 1]);
                    if (!std::isfinite(m[i].real()) || !std::isfinite(m[i].imag()))
                        fail(STN_E_INVALID, where_site(si) + ": non-finite Kraus entry");
                }
                K.push_back(m);
            }
            break;
    }
    // completeness: sum_j K_j^dagger K_j = I
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            cd s = 0;
            for (auto& M : K)
                for (int c = 0; c < d; ++c) s += std::conj(M[c * d + a]) * M[c * d + b];
            if (std::abs(s - (a == b ? 1.0 : 0.0)) > 1e-12)
                fail(STN_E_INVALID, where_site(si) + ": Kraus operators are not trace preserving");
        }
    r.J = (uint32_t)K.size();
    r.q = selection_probs(ch, K, d);
    r.T = thresholds(r.q);
    r.ops.assign(r.J * d * d, 0);
    r.px.assign(r.J, 0);
    r.pz.assign(r.J, 0);
    r.pauli = true;
    for (uint32_t j = 0; j < r.J; ++j) {
        if (r.q[j] > 0) {
            const double sc = 1.0 / std::sqrt(r.q[j]);
            for (int i = 0; i < d * d; ++i) r.ops[j * d * d + i] = K[j][i] * sc;
        }
        uint64_t xm = 0, zm = 0;
        if (!labels.empty()) {
            auto put = [&](int a, uint32_t q) {
                if (a == 1 || a == 2) xm |= 1ull << q;
                if (a == 2 || a == 3) zm |= 1ull << q;
            };
            put(labels[j].first, r.q0);
            if (r.nq == 2) put(labels[j].second, r.q1);
        } else if (r.q[j] > 0) {
            std::vector<cd> op(r.ops.begin() + j * d * d, r.ops.begin() + (j + 1) * d * d);
            if (!as_pauli(op, r.nq, r.q0, r.q1, xm, zm)) r.pauli = false;
        }
        r.px[j] = xm;
        r.pz[j] = zm;
    }
}

bool is_identity(const cd* m, int d) {
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            if (std::abs(m[i * d + j] - (i == j ? 1.0 : 0.0)) > 0) return false;
    return true;
}

void build_lds_program(stn_plan* p) {
    p->lds_ops.clear();
    p->lds_vals.clear();
    p->site_ops.clear();
    p->site_op_off.clear();
    auto push_vals = [&](const std::vector<cd>& v) {
        uint32_t off = (uint32_t)p->lds_vals.size();
        p->lds_vals.insert(p->lds_vals.end(), v.begin(), v.end());
        return off;
    };
    // operator descriptors of every (site, j)
    for (auto& s : p->sites) {
        p->site_op_off.push_back((uint32_t)p->site_ops.size());
        const int d = 1 << s.nq;
        for (uint32_t j = 0; j < s.J; ++j) {
            LdsOp op{};
            op.q0 = s.q0;
            op.q1 = s.q1;
            const cd* m = s.ops.data() + j * d * d;
            if (s.q[j] <= 0 || is_identity(m, d)) {
                op.kind = OP_IDENT;
            } else if (s.pauli) {
                op.kind = OP_PAULI;
                op.xmask = s.px[j];
                op.zmask = s.pz[j];
                if (op.xmask == 0 && op.zmask == 0) op.kind = OP_IDENT;
            } else {
                op.kind = s.nq == 1 ? OP_DENSE1 : OP_DENSE2;
                op.mat = push_vals(std::vector<cd>(m, m + d * d));
            }
            p->site_ops.push_back(op);
        }
    }
    p->site_op_off.push_back((uint32_t)p->site_ops.size());
    size_t si = 0;
    for (uint32_t gi = 0; gi < p->gates.size(); ++gi) {
        const GateRec& g = p->gates[gi];
        LdsOp op{};
        op.q0 = g.q0;
        op.q1 = g.q1;
        switch (g.kind) {
            case STN_G_X: op.kind = OP_PAULI; op.xmask = 1ull << g.q0; break;
            case STN_G_Y: op.kind = OP_PAULI; op.xmask = op.zmask = 1ull << g.q0; break;
            case STN_G_Z: op.kind = OP_PAULI; op.zmask = 1ull << g.q0; break;
            case STN_G_RZ: op.kind = OP_DIAG1; op.mat = push_vals({g.m[0], g.m[3]}); break;
            case STN_G_ZZ: op.kind = OP_DIAG2; op.mat = push_vals({g.m[0], g.m[5], g.m[10], g.m[15]}); break;
            case STN_G_CX:
            case STN_G_U2: op.kind = OP_DENSE2; op.mat = push_vals(g.m); break;
            default: op.kind = OP_DENSE1; op.mat = push_vals(g.m); break;
        }
        p->lds_ops.push_back(op);
        for (; si < p->sites.size() && p->sites[si].gate == gi; ++si) {
            LdsOp so{};
            so.kind = OP_SITE;
            so.site = (uint32_t)si;
            p->lds_ops.push_back(so);
        }
    }
}

// QAOA-structured lowering for the tiled statevector path.  Returns false
// (with a reason) when the circuit does not have the structure.
bool build_tiled(stn_plan* p, std::string& why) {
    const uint32_t n = p->n;
    if (!p->frame_ok) { why = "noise is not Pauli or a non-rotation gate follows a noise site"; return false; }
    if (n > 32) { why = "more than 32 qubits"; return false; }
    if (p->gates.size() < n) { why = "no Hadamard prefix"; return false; }
    uint64_t seen = 0;
    for (uint32_t g = 0; g < n; ++g) {
        if (p->gates[g].kind != STN_G_H || (seen >> p->gates[g].q0) & 1) { why = "circuit does not start with H on every qubit"; return false; }
        seen |= 1ull << p->gates[g].q0;
    }
    p->layers.clear();
    uint32_t g = n;
    while (g < p->gates.size()) {
        TiledLayer L;
        L.rx_gate.assign(n, -1);
        for (; g < p->gates.size() && p->gates[g].kind == STN_G_ZZ; ++g) L.zz_gates.push_back(g);
        for (; g < p->gates.size() && p->gates[g].kind == STN_G_RX; ++g) {
            if (L.rx_gate[p->gates[g].q0] >= 0) break;
            L.rx_gate[p->gates[g].q0] = (int32_t)g;
        }
        // every rotation in the form c [[1, -i t], [-i t, 1]] with |t| <= 1:
        // rx(theta) = -i X rx(theta - pi) when |sin(theta/2)| > |cos(theta/2)|
        for (int32_t gi : L.rx_gate) {
            if (gi < 0) continue;
            GateRec& r = p->gates[gi];
            const double c = std::cos(r.theta / 2), s = std::sin(r.theta / 2);
            r.theta_eff = r.theta;
            r.det_x = 0;
            if (std::abs(s) > std::abs(c)) {
                r.theta_eff = r.theta - M_PI;
                r.det_x = 1ull << r.q0;
            }
        }
        if (L.zz_gates.empty() && std::all_of(L.rx_gate.begin(), L.rx_gate.end(), [](int32_t v) { return v < 0; })) {
            why = "gate " + std::to_string(g) + " is neither zz nor rx";
            return false;
        }
        // zz angles as integer multiples of one base angle per layer
        double base = 0;
        for (uint32_t gi : L.zz_gates)
            if (std::abs(p->gates[gi].theta) > 0) { base = std::abs(p->gates[gi].theta); break; }
        L.base_angle = base;
        L.mult_sum = 0;
        for (uint32_t gi : L.zz_gates) {
            const double t = p->gates[gi].theta;
            const double mr = base > 0 ? std::round(t / base) : 0.0;
            if (std::abs(t - mr * base) > 1e-12 * std::max(1.0, std::abs(t)) || std::abs(mr) > 16) {
                why = "zz angles of a layer are not small integer multiples of one angle";
                return false;
            }
            L.zz_mult.push_back((int32_t)mr);
            L.mult_sum += (int32_t)std::abs(mr);
        }
        p->layers.push_back(L);
    }
    return true;
}

}  // namespace

// Whether a tiled plan keeps half the amplitudes.  Every circuit
// of the tiled lowering (H on every qubit, zz and rx gates with the signs
// the Pauli frame sets) commutes with X on all qubits and |+>^n is fixed by
// it, so every trajectory has psi(~z) = psi(z); the ZZ observable takes the
// same value at z and ~z.  The kernels then store the amplitudes with qubit
// n-1 = 0 and read psi(z', 1) at ~z'.  A tile must fit in the stored
// qubits with one fixed bit left: n >= tile bits + 1 for the complex64
// tiles, n >= 13 for the 12-qubit complex128 ones.
static bool tiled_half(const stn_plan* p) {
    return p->n >= (p->opts.precision == 64 ? p->tile_bits + 1 : 13u) && !p->opts.sv_full_state;
}

// Qubits per tile.  complex64: 15-qubit tiles (a 1024-thread workgroup per
// CU) leave the strided tile 4 low storage bits up to n = 26 (128-byte runs,
// whole lines), where 14-qubit tiles leave 3 at n = 25 and 2 at n = 26.
// Up to n = 24 the 14-qubit tiles keep 128-byte runs too, and their two
// resident workgroups per CU overlap one's memory traffic with the other's
// exchanges, which makes their contiguous passes faster.
static uint32_t tiled_tile_bits(const stn_plan* p) {
    if (p->opts.precision == 128) return tiled128_tile_bits();
    if (p->opts.sv_tile_bits) return p->opts.sv_tile_bits;
    return p->n >= 25 ? 15u : 14u;
}

// low storage bits every tile after the first keeps: two tiles of 15 qubits
// cover 30 - coal qubits (n counts qubit n-1 of a half-state plan), so
// n = 27 and 28 keep two tiles per layer with 3 and 2; from n = 29 a layer
// needs three tiles anyway, and all of them keep 4 (whole 128-byte lines)
static uint32_t tiled_coal(const stn_plan* p) {
    if (p->opts.precision == 128) return 3;
    if (p->tile_bits == 14) return 2;
    return (p->n == 27 || p->n == 28) ? 30u - p->n : 4u;
}

// Pass schedule of the tiled lowering.  A layer's rotations are split over
// tiles: the first holds the low `tile_bits` storage bits, the next ones
// `coal` low bits (coalescing) plus the next high qubits.  Rotations on
// different qubits commute, so the tiles of a layer may be visited in any
// order; visiting them in alternating order (forward for even layers,
// backward for odd ones) makes the last tile of a layer and the first tile of
// the next one the same, and those two become one pass: rotate (layer l),
// diagonal (layer l+1), rotate (layer l+1).  p layers on k tiles cost
// p (k - 1) + 1 passes instead of p k.
void schedule_tiled(stn_plan* p, uint32_t tile_bits, uint32_t coal) {
    const uint32_t n = p->n;
    p->passes.clear();
    std::vector<uint32_t> tiles;
    const uint32_t q = std::min(n, tile_bits);
    tiles.push_back((q == 32 ? 0u : (1u << q)) - 1u);
    for (uint32_t lo = q; lo < n;) {
        const uint32_t take = std::min(n - lo, q - coal);
        uint32_t m = (1u << coal) - 1u;
        for (uint32_t b = lo; b < lo + take; ++b) m |= 1u << b;
        // fill the tile up to q bits with passenger bits just above the coalescing bits
        for (uint32_t b = coal; __builtin_popcount(m) < (int)q && b < n; ++b) m |= 1u << b;
        tiles.push_back(m);
        lo += take;
    }
    struct Op { int32_t layer; uint32_t tile; uint32_t mask; bool first; };
    std::vector<Op> ops;
    const uint32_t k = (uint32_t)tiles.size();
    // 15-qubit complex64 tiles whose strided tiles read whole 128-byte lines
    // start with the last tile: the generating and the reducing pass are
    // then strided and the read/write passes on the contiguous tile become
    // one more (shorter runs make strided writes without the line's reads
    // costly, so n = 27, 28 keep the contiguous tile first)
    const bool strided_first = p->opts.precision == 64 && tile_bits == 15 && k >= 2 && coal >= 4;
    for (uint32_t l = 0; l < p->layers.size(); ++l) {
        uint32_t mixed = 0;
        for (uint32_t i = 0; i < k; ++i) {
            const uint32_t t = ((l % 2 == 0) != strided_first) ? i : k - 1 - i;
            uint32_t mm = 0;
            for (uint32_t qb = 0; qb < n; ++qb)
                if (((tiles[t] >> qb) & 1) && !((mixed >> qb) & 1) && p->layers[l].rx_gate[qb] >= 0) mm |= 1u << qb;
            mixed |= tiles[t];
            if (i > 0 && mm == 0) continue;
            ops.push_back({(int32_t)l, t, mm, i == 0});
        }
    }
    for (const Op& o : ops) {
        if (!p->passes.empty()) {
            TiledPass& b = p->passes.back();
            if (o.first && b.mix2 < 0 && b.mix1 == o.layer - 1 && b.tile_mask == tiles[o.tile]) {
                b.diag_b = o.layer;
                b.mix2 = o.layer;
                b.mix2_mask = o.mask;
                continue;
            }
        }
        TiledPass ps;
        ps.tile_mask = tiles[o.tile];
        ps.diag_a = o.first ? o.layer : -1;
        ps.mix1 = o.layer;
        ps.mix1_mask = o.mask;
        p->passes.push_back(ps);
    }
    if (p->passes.empty()) {
        TiledPass ps;
        ps.tile_mask = tiles[0];
        p->passes.push_back(ps);
    }
    p->passes.front().init = true;
    p->passes.back().last = true;
}

void build_plan(stn_plan* p, const stn_circuit* c, const stn_noise_model* nm, const stn_observable* ob) {
    if (!c) fail(STN_E_INVALID, "circuit is NULL");
    if (c->n_qubits < 1 || c->n_qubits > 64) fail(STN_E_INVALID, "n_qubits must be in 1..64");
    if (c->n_gates > 0 && !c->gates) fail(STN_E_INVALID, "gates is NULL");
    const uint32_t n = c->n_qubits;
    p->n = n;
    p->gates.resize(c->n_gates);
    for (uint32_t i = 0; i < c->n_gates; ++i) gate_record(p->gates[i], c->gates[i], n, i);
    const uint32_t S = nm ? nm->n_channels : 0;
    if (S > 0 && !nm->channels) fail(STN_E_INVALID, "channels is NULL");
    p->sites.resize(S);
    for (uint32_t s = 0; s < S; ++s) {
        if (s > 0 && nm->channels[s].after_gate < nm->channels[s - 1].after_gate)
            fail(STN_E_INVALID, where_site(s) + ": channels must be ordered by after_gate");
        site_record(p->sites[s], nm->channels[s], n, c->n_gates, s);
    }
    if (ob && ob->n_terms > 0) {
        if (!ob->uv || !ob->w) fail(STN_E_INVALID, "observable arrays are NULL");
        for (uint32_t t = 0; t < ob->n_terms; ++t) {
            const uint32_t u = ob->uv[2 * t], v = ob->uv[2 * t + 1];
            if (u >= n || v >= n || u == v) fail(STN_E_INVALID, "observable term " + std::to_string(t) + ": bad qubits");
            if (!std::isfinite(ob->w[t])) fail(STN_E_INVALID, "observable term " + std::to_string(t) + ": bad weight");
            p->obs_u.push_back(u);
            p->obs_v.push_back(v);
            p->obs_w.push_back(ob->w[t]);
        }
    }
    // Pauli frame: all sites Pauli, and every gate that is not a Pauli rotation
    // or a Pauli acts on qubits no earlier site touched.
    p->frame_ok = true;
    {
        uint64_t touched = 0;
        size_t si = 0;
        for (uint32_t gi = 0; gi < p->gates.size(); ++gi) {
            const GateRec& g = p->gates[gi];
            const uint64_t qm = (1ull << g.q0) | (g.nq == 2 ? (1ull << g.q1) : 0);
            const bool pauli_gate = g.kind == STN_G_X || g.kind == STN_G_Y || g.kind == STN_G_Z;
            if (!g.rotation && !pauli_gate && (touched & qm)) p->frame_ok = false;
            for (; si < p->sites.size() && p->sites[si].gate == gi; ++si) {
                const SiteRec& s = p->sites[si];
                if (!s.pauli) p->frame_ok = false;
                touched |= (1ull << s.q0) | (s.nq == 2 ? (1ull << s.q1) : 0);
            }
        }
    }
    const uint32_t outs = p->opts.outputs;
    if ((outs & STN_OUT_ENERGY) && !ob) fail(STN_E_INVALID, "ENERGY output requested without an observable");
    const bool dense_out = outs & (STN_OUT_RHO | STN_OUT_DIAG | STN_OUT_STATES);
    const uint32_t lds_max = p->opts.precision == 128 ? 12 : 13;
    std::string why;
    uint32_t kind = p->opts.plan_kind;
    if (kind == STN_PLAN_AUTO) {
        if (n <= lds_max) {
            kind = STN_PLAN_SV_LDS;
        } else if (dense_out) {
            // sigma alone is kept by the gate-by-gate lowering; rho_hat and states need LDS sizes
            if ((outs & (STN_OUT_RHO | STN_OUT_STATES)) || n > kGatesMaxQubits)
                fail(STN_E_UNSUPPORTED, "rho_hat / state outputs need n <= " + std::to_string(lds_max) +
                                            " (sigma alone: n <= 30)");
            kind = STN_PLAN_SV_GATES;
        } else {
            // statevector passes vs lightcone networks: estimated seconds per trajectory
            // (HBM-bound passes; lightcone networks: their own estimate)
            double sv_t = -1, tn_t = -1;
            const bool c128 = p->opts.precision == 128;
            p->tile_bits = tiled_tile_bits(p);
            if (n >= (c128 ? 13u : p->tile_bits) && build_tiled(p, why)) {
                schedule_tiled(p, p->tile_bits, tiled_coal(p));
                double bytes = 0;
                const int stored = (int)n - (tiled_half(p) ? 1 : 0);
                for (auto& ps : p->passes)
                    bytes += std::ldexp(c128 ? 16.0 : 8.0, stored) * ((ps.init ? 0 : 1) + (ps.last ? 0 : 1));
                // measured: about 5 TB/s while the strided tiles keep runs of
                // 128 bytes or more (n <= 24), about 3 TB/s at n = 26
                sv_t = bytes / (n <= 24 ? 5e12 : 3e12);
            }
            // below half a microsecond per trajectory (a few ms of device
            // time for thousands of trajectories) the networks cannot save
            // what building them costs (milliseconds per observable term)
            constexpr double kNetworksWorthSeconds = 0.5e-6;
            if (sv_t < 0 || sv_t >= kNetworksWorthSeconds) {
                try {
                    build_lightcone(p);
                    tn_t = p->lc_est_s;
                } catch (const Error& e) {
                    if (e.status != STN_E_UNSUPPORTED) throw;
                    if (why.empty()) why = e.msg;
                    else why += "; " + e.msg;
                }
            }
            if (tn_t >= 0 && (sv_t < 0 || tn_t < sv_t)) kind = STN_PLAN_LIGHTCONE;
            else if (sv_t >= 0) kind = STN_PLAN_SV_TILED;
            else if (n <= kGatesMaxQubits) kind = STN_PLAN_SV_GATES;   // any circuit and channel
            else fail(STN_E_UNSUPPORTED, "no lowering for this circuit: " + why);
            if (kind != STN_PLAN_LIGHTCONE && p->lc && p->lc_free) {
                p->lc_free(p->lc);
                p->lc = nullptr;
            }
            if (kind == STN_PLAN_LIGHTCONE) {
                // the networks use the gates as given: undo the tiled rewrite
                for (auto& g : p->gates) {
                    g.det_x = 0;
                    g.theta_eff = g.theta;
                }
                p->passes.clear();
            }
        }
    }
    if (kind == STN_PLAN_SV_LDS) {
        if (n > lds_max) fail(STN_E_UNSUPPORTED, "whole-state-in-LDS lowering needs n <= " + std::to_string(lds_max));
        build_lds_program(p);
    } else if (kind == STN_PLAN_SV_TILED) {
        if (dense_out) fail(STN_E_UNSUPPORTED, "the tiled lowering produces energies only");
        const bool c128 = p->opts.precision == 128;
        p->tile_bits = tiled_tile_bits(p);
        if (n < p->tile_bits)
            fail(STN_E_UNSUPPORTED, "the tiled lowering with " + std::to_string(p->tile_bits) +
                                        "-qubit tiles needs n >= " + std::to_string(p->tile_bits));
        if (p->layers.empty() && !build_tiled(p, why)) fail(STN_E_UNSUPPORTED, "tiled lowering: " + why);
        if (c128) {
            // the complex128 kernels apply every rx as given
            for (auto& g : p->gates) {
                g.det_x = 0;
                g.theta_eff = g.theta;
            }
        }
        schedule_tiled(p, p->tile_bits, tiled_coal(p));
        p->sv_half = tiled_half(p);
    } else if (kind == STN_PLAN_LIGHTCONE) {
        if (dense_out) fail(STN_E_UNSUPPORTED, "the lightcone lowering produces energies only");
        if (!p->lc) build_lightcone(p);
    } else if (kind == STN_PLAN_SV_GATES) {
        if (outs & (STN_OUT_RHO | STN_OUT_STATES))
            fail(STN_E_UNSUPPORTED, "the gate-by-gate lowering keeps energies and sigma only");
        if (n < 2 || n > kGatesMaxQubits) fail(STN_E_UNSUPPORTED, "the gate-by-gate lowering needs 2 <= n <= 30");
        if (p->lc && p->lc_free) {
            p->lc_free(p->lc);
            p->lc = nullptr;
        }
        for (auto& g : p->gates) {   // gates as given (no Pauli-frame rewrite)
            g.det_x = 0;
            g.theta_eff = g.theta;
        }
        p->passes.clear();
        build_lds_program(p);
        build_gate_groups(p);
    } else {
        fail(STN_E_INVALID, "unknown plan kind");
    }
    p->kind = kind;
    // launch shape before any tuning: for the 14-qubit complex64 tiles, two
    // resident workgroups per CU (variant 2), the autotuner's choice on every
    // size measured; the 15-qubit tiles have one shape
    if (kind == STN_PLAN_SV_TILED && p->opts.precision == 64) p->variant = p->tile_bits == 15 ? 0 : 2;
    // cost model and batch size
    const double elem = p->opts.precision == 128 ? 16.0 : 8.0;
    const double N = std::ldexp(1.0, (int)n);
    if (kind == STN_PLAN_SV_LDS) {
        p->width = n;
        p->bytes_per_traj = (dense_out ? N * elem : 0) + 8.0;
        double fl = 0;
        for (auto& g : p->gates) fl += (g.nq == 1 ? 8.0 : 32.0) * N;
        p->flops_per_traj = fl;
        const double per = (dense_out ? N * elem : 0) + 64.0 + p->sites.size();
        const double budget = p->opts.hbm_budget ? (double)p->opts.hbm_budget : 64.0 * (1ull << 30);
        p->max_batch = p->opts.max_batch ? p->opts.max_batch : (uint32_t)std::min(65535.0, std::max(1.0, budget / per));
        p->peak_bytes = per * p->max_batch;
    } else if (kind == STN_PLAN_SV_GATES) {
        // every fused group reads and writes the state once (the first only
        // writes), and the energy reads it
        p->width = n;
        double fl = 0;
        for (auto& o : p->lds_ops) {
            if (o.kind == OP_IDENT) continue;
            const bool two = o.kind == OP_DENSE2 || o.kind == OP_DIAG2 || (o.kind == OP_SITE && p->sites[o.site].nq == 2);
            fl += (two ? 32.0 : 8.0) * N;
        }
        p->n_passes = (uint32_t)p->gate_groups.size();
        p->bytes_per_traj = N * elem * 2.0 * (double)p->gate_groups.size();
        p->flops_per_traj = fl;
        const double per = N * elem + 64.0 * 8.0 + 64.0 + p->sites.size();
        const double budget = p->opts.hbm_budget ? (double)p->opts.hbm_budget : 64.0 * (1ull << 30);
        p->max_batch = p->opts.max_batch ? p->opts.max_batch : (uint32_t)std::max(1.0, std::min(4096.0, std::floor(budget / per)));
        p->peak_bytes = per * p->max_batch;
    } else if (kind == STN_PLAN_LIGHTCONE) {
        // width / steps / flops / bytes set by build_lightcone
        p->max_batch = p->opts.max_batch ? p->opts.max_batch : 65535;
        p->peak_bytes = (double)p->max_batch * (p->obs_u.size() * 8.0 + 64.0 + p->sites.size()) + p->lc_arena_bytes;
    } else {
        p->width = n;
        p->n_passes = (uint32_t)p->passes.size();
        double bytes = 0, fl = 0;
        const double Ns = p->sv_half ? N / 2 : N;   // amplitudes stored (and updated) per trajectory
        for (auto& ps : p->passes) {
            bytes += (ps.init ? 0 : Ns * elem) + (ps.last ? 0 : Ns * elem);
            fl += Ns * 6.0 * (__builtin_popcount(ps.mix1_mask) + __builtin_popcount(ps.mix2_mask)) +
                  Ns * 6.0 * ((ps.diag_a >= 0) + (ps.diag_b >= 0)) + (ps.last ? Ns * 4.0 : 0);
        }
        p->bytes_per_traj = bytes;
        p->flops_per_traj = fl;
        const double per = Ns * elem + 64.0 * 1024;
        const double budget = p->opts.hbm_budget ? (double)p->opts.hbm_budget : 64.0 * (1ull << 30);
        p->max_batch = p->opts.max_batch ? p->opts.max_batch : (uint32_t)std::max(1.0, std::min(4096.0, std::floor(budget / per)));
        p->peak_bytes = per * p->max_batch;
    }
}

}  // namespace stn
