// Device copies of the plan tables (noise sites, gate generators, observable,
// and the lowering-specific programs).  Complex values are computed on the
// host in binary64 and rounded once to the contraction precision.
#include <cmath>

#include "stn_internal.h"

namespace stn {

namespace {
template <class T>
void up(DevBuf& d, const Allocator* a, const std::vector<T>& v, hipStream_t s) {
    upload(d, a, v.data(), v.size() * sizeof(T), s);
}

void up_complex(DevBuf& d32, DevBuf& d64, const Allocator* a, const std::vector<cd>& v, hipStream_t s) {
    std::vector<float> f(2 * v.size() + 2);
    std::vector<double> g(2 * v.size() + 2);
    for (size_t i = 0; i < v.size(); ++i) {
        f[2 * i] = (float)v[i].real();
        f[2 * i + 1] = (float)v[i].imag();
        g[2 * i] = v[i].real();
        g[2 * i + 1] = v[i].imag();
    }
    up(d32, a, f, s);
    up(d64, a, g, s);
}
}  // namespace

void upload_plan_tables(stn_plan* p, hipStream_t s) {
    const Allocator* a = &p->alloc;
    std::vector<uint64_t> T, px, pz;
    std::vector<uint32_t> off, sg;
    for (auto& st : p->sites) {
        off.push_back((uint32_t)T.size());
        T.insert(T.end(), st.T.begin(), st.T.end());
        px.insert(px.end(), st.px.begin(), st.px.end());
        pz.insert(pz.end(), st.pz.begin(), st.pz.end());
        sg.push_back(st.gate);
    }
    off.push_back((uint32_t)T.size());
    T.push_back(0);
    px.push_back(0);
    pz.push_back(0);
    sg.push_back(0);
    up(p->d_site_T, a, T, s);
    up(p->d_site_off, a, off, s);
    up(p->d_site_gate, a, sg, s);
    up(p->d_site_px, a, px, s);
    up(p->d_site_pz, a, pz, s);
    std::vector<uint64_t> gx, gz, dx;
    for (auto& g : p->gates) {
        gx.push_back(g.rotation ? g.gx : 0);
        gz.push_back(g.rotation ? g.gz : 0);
        dx.push_back(g.det_x);
    }
    gx.push_back(0);
    gz.push_back(0);
    dx.push_back(0);
    up(p->d_gate_gx, a, gx, s);
    up(p->d_gate_gz, a, gz, s);
    up(p->d_gate_dx, a, dx, s);
    std::vector<uint32_t> uv;
    for (size_t t = 0; t < p->obs_u.size(); ++t) {
        uv.push_back(p->obs_u[t]);
        uv.push_back(p->obs_v[t]);
    }
    uv.push_back(0);
    uv.push_back(0);
    std::vector<double> w = p->obs_w;
    w.push_back(0);
    up(p->d_obs, a, uv, s);
    up(p->d_obs_w, a, w, s);
    {
        // terms per qubit (each term under both of its qubits)
        std::vector<uint32_t> adj(p->n + 1, 0), terms;
        for (size_t t = 0; t < p->obs_u.size(); ++t) {
            adj[p->obs_u[t] + 1]++;
            adj[p->obs_v[t] + 1]++;
        }
        for (uint32_t q = 0; q < p->n; ++q) adj[q + 1] += adj[q];
        terms.resize(adj[p->n]);
        std::vector<uint32_t> fill(adj.begin(), adj.end() - 1);
        for (size_t t = 0; t < p->obs_u.size(); ++t) {
            terms[fill[p->obs_u[t]]++] = (uint32_t)t;
            terms[fill[p->obs_v[t]]++] = (uint32_t)t;
        }
        adj.insert(adj.end(), terms.begin(), terms.end());
        up(p->d_obs_adj, a, adj, s);
    }

    if (p->kind == STN_PLAN_SV_LDS || p->kind == STN_PLAN_SV_GATES) {
        std::vector<LdsOp> ops = p->lds_ops, sops = p->site_ops;
        ops.push_back(LdsOp{});
        sops.push_back(LdsOp{});
        up(p->d_lds_ops, a, ops, s);
        up(p->d_site_ops, a, sops, s);
        up(p->d_site_op_off, a, p->site_op_off, s);
        up_complex(p->d_lds_vals32, p->d_lds_vals64, a, p->lds_vals, s);
        if (p->kind == STN_PLAN_SV_GATES) upload_gate_groups(p, s);
    } else if (p->kind == STN_PLAN_SV_TILED) {
        if (p->opts.precision == 128) upload_tiled128(p, s);
        else upload_tiled(p, s);
    } else if (p->kind == STN_PLAN_LIGHTCONE) {
        upload_lightcone(p, s);
    }
}

}  // namespace stn
