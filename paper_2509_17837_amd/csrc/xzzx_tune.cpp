// Autotuner of the annealing launch knobs.  Every candidate computes the
// same chains bit for bit, so the choice only affects speed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <random>
#include <vector>

#include "xzzx_internal.h"

using namespace xzzx;

namespace {

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
    int alloc(size_t n)
    {
        if (hipMalloc(&p, n ? n : 1) != hipSuccess) { p = nullptr; set_error("autotune allocation"); return XZZX_ENOMEM; }
        return XZZX_OK;
    }
    template <typename T> T *as() { return static_cast<T *>(p); }
};

}  // namespace

extern "C" int xzzx_plan_autotune(xzzx_plan *plan, int n_rep, int n_syn, int probe_sweeps, void *stream,
                                  xzzx_tune_result *out)
{
    if (!plan || n_rep < 1 || n_syn < 1 || probe_sweeps < 1) { set_error("bad autotune arguments"); return XZZX_EINVAL; }
    Plan &P = plan->P;
    if (P.order || P.ladder_k) {
        // the random-site and ladder kernels have no knobs
        if (out) {
            out->kernel = P.order ? XZZX_KERNEL_SITE : XZZX_KERNEL_LADDER;
            out->lanes_per_chain = 1;
            for (float &t : out->times_ms) t = -1.0f;
        }
        return XZZX_OK;
    }
    const int sweeps = std::min(probe_sweeps, std::max(P.n_sweeps, 1));
    std::vector<double> beta(P.beta.begin(), P.beta.begin() + std::min<size_t>(sweeps, P.beta.size()));
    while ((int)beta.size() < sweeps) beta.push_back(1.0);
    xzzx_lattice lat;
    lat.L = P.lat;
    xzzx_plan *probe = nullptr;
    int rc = xzzx_plan_create(&lat, P.W, P.Wg, beta.data(), sweeps, &probe);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int nq = P.lat.nq, ns = P.lat.nstab;
    // random syndromes (every bit pattern is a valid syndrome)
    std::mt19937 gen(12345u);
    std::vector<uint8_t> syn((size_t)n_syn * ns);
    for (auto &b : syn) b = (uint8_t)(gen() & 1u);
    std::vector<uint32_t> uid(n_syn);
    for (int i = 0; i < n_syn; ++i) uid[i] = (uint32_t)i;
    DevBuf d_syn, d_uid, d_out, d_ws;
    const size_t nc = (size_t)n_syn * 4 * n_rep;
    if ((rc = d_syn.alloc(syn.size())) || (rc = d_uid.alloc(4 * uid.size())) ||
        (rc = d_out.alloc(4 * (size_t)n_syn + n_syn + (size_t)n_syn * nq + 64))) {
        xzzx_plan_destroy(probe);
        return rc;
    }
    (void)hipMemcpy(d_syn.p, syn.data(), syn.size(), hipMemcpyHostToDevice);
    (void)hipMemcpy(d_uid.p, uid.data(), 4 * uid.size(), hipMemcpyHostToDevice);
    xzzx_group g{};
    g.plan = probe;
    g.n_syn = n_syn;
    g.n_rep = n_rep;
    g.d_uid = d_uid.as<uint32_t>();
    g.d_syn = d_syn.as<uint8_t>();
    g.d_e_best = d_out.as<int32_t>();
    g.d_cls = d_out.as<uint8_t>() + 4 * (size_t)n_syn;
    g.d_recovery = d_out.as<uint8_t>() + 5 * (size_t)n_syn;
    size_t wsb = 0;
    rc = xzzx_decode_workspace(&g, 1, &wsb);
    if (!rc) rc = d_ws.alloc(wsb);
    if (!rc) rc = xzzx_decode(&g, 1, 1, 2, XZZX_GREEDY_RANDOM, XZZX_FLAG_STAGE_GREEDY, d_ws.p, wsb, stream);
    (void)nc;
    float times[8];
    for (float &t : times) t = -1.f;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) { set_error("events"); rc = XZZX_EDEVICE; }
    for (int cand = 0; cand < 8 && !rc; ++cand) {
        if (cand == 0) {
            if (!P.row_words && !P.static_ok) continue;
            probe->P.use_rows = 1;
        } else {
            const int lanes = 1 << (cand - 1);
            if (probe->P.lds_bytes_anneal(lanes) > 65536) continue;
            if ((rc = xzzx_plan_set_lanes(probe, lanes))) break;
        }
        float best = -1.f;
        for (int rep = 0; rep < 4 && !rc; ++rep) {
            (void)hipEventRecord(e0, s);
            rc = xzzx_decode(&g, 1, 1, 2, XZZX_GREEDY_RANDOM, XZZX_FLAG_STAGE_ANNEAL, d_ws.p, wsb, stream);
            (void)hipEventRecord(e1, s);
            if (rc) break;
            if (hipEventSynchronize(e1) != hipSuccess) { set_error("autotune run failed"); rc = XZZX_EDEVICE; break; }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0 && (best < 0.f || ms < best)) best = ms;   // first run warms up
        }
        times[cand] = best;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    xzzx_plan_destroy(probe);
    if (rc) return rc;
    int pick = -1;
    for (int c = 0; c < 8; ++c)
        if (times[c] >= 0.f && (pick < 0 || times[c] < times[pick])) pick = c;
    if (pick < 0) { set_error("no autotune candidate ran"); return XZZX_ERANGE; }
    if (pick == 0) {
        rc = xzzx_plan_set_kernel(plan, XZZX_KERNEL_ROWS);
    } else {
        rc = xzzx_plan_set_lanes(plan, 1 << (pick - 1));
    }
    if (rc) return rc;
    if (out) {
        out->kernel = !P.use_rows ? XZZX_KERNEL_BYTES
                      : (P.static_d || P.planar_d) ? XZZX_KERNEL_ROWS : XZZX_KERNEL_ROWS_GENERIC;
        out->lanes_per_chain = P.lanes;
        std::memcpy(out->times_ms, times, sizeof(times));
    }
    return XZZX_OK;
}
