// Serving loop: continuous batching of single-syndrome decode requests.
//
// A scheduler thread owns one HIP stream (default priority) and repeats:
//   1. admit queued requests into free device slots while the LDS budget
//      allows (greedy references for all admissions of the slice, batched per
//      plan, written straight into the slots);
//   2. advance every resident request by its share of sweeps (balanced so
//      that every task carries about the same sequential work), with as many
//      lanes per chain as the load allows: one task per group of chains, one
//      launch per kernel family and distance, the launches of a slice running
//      concurrently;
//   3. finish requests whose schedule is complete (per-coset reduction and
//      replay of the best chain on the device; results gathered on the
//      device and copied to pinned host memory in one transfer);
//   4. wait for the slice, then publish finished results with their latency.
// Requests that arrive while a slice runs join at the next slice boundary.
// Admission may hold more tasks than the device runs at once (the default
// LDS budget is four devices' worth): the hardware dispatcher then starts
// queued tasks as earlier ones end, so a slice's short tasks do not leave
// their waves idle until the slice's longest task is done.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "xzzx_internal.h"

using namespace xzzx;

namespace {

using Clock = std::chrono::steady_clock;

struct Pending {
    uint64_t ticket;
    const xzzx_plan *plan;
    std::vector<uint8_t> syn;
    uint32_t uid;
    int n_rep;
    Clock::time_point submit;
};

struct Slot {
    bool busy = false;
    uint64_t ticket = 0;
    const Plan *plan = nullptr;
    uint32_t uid = 0;
    int n_rep = 0;
    int t = 0;             // sweeps done
    bool started = false;  // first slice launched
    size_t lds = 0;        // LDS its tasks take
    Clock::time_point submit, admit;
};

struct Done {
    int32_t e_best, cls, e_cls[4];
    std::vector<uint8_t> recovery;
    double latency_s, queue_s;
};

}  // namespace

struct xzzx_server {
    xzzx_server_cfg cfg{};
    int device = 0;
    hipStream_t stream = nullptr;
    // device slot pool
    uint8_t *d_pool = nullptr;
    size_t slot_bytes = 0, off_refs = 0, off_states = 0, off_e3 = 0, off_qraw = 0, off_res = 0, off_rec = 0;
    size_t off_cp = 0, off_cpk = 0, off_cpm = 0;   // kept states: bytes [2][4R][nq], packed rows [2][4R][cpk_words], entries [4R]
    int cpk_words = 0;
    // staging (device + pinned host)
    uint8_t *d_stage = nullptr, *h_stage = nullptr;
    size_t stage_bytes = 0, st_syn = 0, st_uid = 0, st_map = 0, st_tasks = 0, st_fin = 0, st_out = 0;
    size_t max_tasks = 0;
    size_t lds_budget = 0, lds_used = 0;
    int64_t wave_budget = 0;
    int max_nstab = 0;
    std::vector<Slot> slots;
    // free slot indices (a stack) and the resident ones (unordered; position
    // of each in resident_pos), so no step scans every slot
    std::vector<int> free_slots, resident, resident_pos;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Pending> pending;
    std::unordered_map<uint64_t, Done> done;
    std::unordered_map<uint64_t, int> where;   // ticket -> 0 queued, 1 resident
    uint64_t next_ticket = 1;
    bool stop = false;
    int error = XZZX_OK;
    std::string error_msg;
    // statistics
    std::vector<double> latencies;
    int64_t submitted = 0, completed = 0, rejected = 0, slices = 0;
    double attempts_done = 0.0;
    bool started = false;
    Clock::time_point first_admit, last_done;

    uint8_t *slot_ptr(int s) { return d_pool + (size_t)s * slot_bytes; }
    // bytes per finished request in the result staging: 32-byte result, recovery, 16-byte aligned
    size_t out_stride() const { return (32 + (size_t)cfg.max_qubits + 15) & ~size_t(15); }
    void run();
    int slice();
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t task_lds(const Plan &P, int *chains_per_task)
{
    if (P.use_rows) {
        *chains_per_task = kWave;
        // the specialised kernels keep rows in registers: LDS holds only their tables
        return P.static_d ? kStaticLdsBytes : P.lds_bytes_rows();
    }
    *chains_per_task = kWave / P.lanes;
    return P.lds_bytes_anneal(P.lanes);
}

// resident requests per additional sweeps_per_slice of a slice
constexpr int64_t kSliceGrowth = 64;

// Philox blocks (four generators each) of a colour class: the byte-state
// kernel gives each lane of a chain whole blocks
int class_blocks(const Plan &P)
{
    return (std::max(1, P.lat.nstab / 4) + 3) / 4;
}

// lanes per chain for a request when the slice offers g: where g lanes can
// take every generator of a colour class, the least power of two that gives
// each lane one generator (the byte-state kernel's one-move-per-lane form);
// else the least power of two that gives every lane at most one block,
// capped at g (more lanes would sit idle)
int lanes_for(const Plan &P, int g)
{
    const int M = std::max(1, P.lat.per_class);
    int c = 1;
    if (M <= g && g >= 4) {
        while (c < M) c *= 2;
        return std::max(c, 4);
    }
    const int nblk = class_blocks(P);
    while (c < nblk && 2 * c <= g) c *= 2;
    return c;
}

// sequential work of one sweep of one chain: attempts on the packed-row
// kernels (g = 1); on the byte-state kernel, in units of half a block per
// lane: one generator per lane measured about half the phase latency of one
// block per lane (0.43-0.47 and 0.92 us at 64 lanes), and each further block
// per lane adds about one block's latency
int64_t sweep_cost(const Plan &P, int g)
{
    if (g == 1) return P.lat.nstab;
    const int gr = lanes_for(P, g);
    if (std::max(1, P.lat.per_class) <= gr && gr >= 4) return 1;
    return 2 * ((class_blocks(P) + gr - 1) / gr);
}

size_t request_lds(const Plan &P, int n_rep)
{
    int C = 1;
    const size_t per = task_lds(P, &C);
    return per * (size_t)((4 * n_rep + C - 1) / C);
}

int check(hipError_t e, const char *what)
{
    if (e == hipSuccess) return XZZX_OK;
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return XZZX_EDEVICE;
}

}  // namespace

int xzzx_server::slice()
{
    // ---- 1. admission -----------------------------------------------------
    std::vector<int> admitted;
    {
        std::lock_guard<std::mutex> lk(mu);
        // admit in arrival order; stage grouped by (plan, n_rep) so that one
        // greedy launch covers every admission of a plan
        std::vector<std::pair<int, Pending>> adm;
        while (!pending.empty()) {
            const Pending &p = pending.front();
            const Plan &P = p.plan->P;
            const size_t need = request_lds(P, p.n_rep);
            if (lds_used + need > lds_budget && lds_used > 0) break;
            if (free_slots.empty()) break;
            const int s = free_slots.back();
            free_slots.pop_back();
            resident_pos[s] = (int)resident.size();
            resident.push_back(s);
            Slot &sl = slots[s];
            sl.busy = true;
            sl.ticket = p.ticket;
            sl.plan = &P;
            sl.uid = p.uid;
            sl.n_rep = p.n_rep;
            sl.t = 0;
            sl.started = false;
            sl.lds = need;
            sl.submit = p.submit;
            sl.admit = Clock::now();
            lds_used += need;
            where[p.ticket] = 1;
            if (!started) { started = true; first_admit = sl.admit; }
            adm.emplace_back(s, std::move(pending.front()));
            pending.pop_front();
        }
        std::stable_sort(adm.begin(), adm.end(), [](const auto &a, const auto &b) {
            if (a.second.plan != b.second.plan) return std::less<const xzzx_plan *>()(a.second.plan, b.second.plan);
            return a.second.n_rep < b.second.n_rep;
        });
        // stage the syndromes (index = position in `admitted`)
        for (const auto &[s, p] : adm) {
            std::memcpy(h_stage + st_syn + admitted.size() * (size_t)max_nstab, p.syn.data(), p.syn.size());
            reinterpret_cast<uint32_t *>(h_stage + st_uid)[admitted.size()] = p.uid;
            reinterpret_cast<int32_t *>(h_stage + st_map)[admitted.size()] = s;
            admitted.push_back(s);
        }
    }
    int rc = XZZX_OK;
    if (!admitted.empty()) {
        const size_t n = admitted.size();
        rc = check(hipMemcpyAsync(d_stage + st_syn, h_stage + st_syn, n * (size_t)max_nstab, hipMemcpyHostToDevice, stream), "stage syndromes");
        if (!rc) rc = check(hipMemcpyAsync(d_stage + st_uid, h_stage + st_uid, n * 4, hipMemcpyHostToDevice, stream), "stage uids");
        if (!rc) rc = check(hipMemcpyAsync(d_stage + st_map, h_stage + st_map, n * 4, hipMemcpyHostToDevice, stream), "stage slots");
        // one greedy launch per (plan, n_rep) over consecutive staged entries;
        // the launches of different plans run concurrently
        std::vector<std::pair<size_t, size_t>> runs;
        for (size_t i = 0; i < n;) {
            size_t j = i + 1;
            const Slot &a = slots[admitted[i]];
            while (j < n && slots[admitted[j]].plan == a.plan && slots[admitted[j]].n_rep == a.n_rep) ++j;
            runs.emplace_back(i, j);
            i = j;
        }
        if (!rc)
            rc = run_concurrently(stream, (int)runs.size(), [&](int r, hipStream_t s) {
                const size_t i = runs[r].first, j = runs[r].second;
                const Slot &a = slots[admitted[i]];
                return serve_greedy(*a.plan, d_stage + st_syn + i * (size_t)max_nstab, max_nstab,
                                    reinterpret_cast<const uint32_t *>(d_stage + st_uid) + i,
                                    reinterpret_cast<const int32_t *>(d_stage + st_map) + i, (int)(j - i), a.n_rep,
                                    d_pool + off_refs, (int64_t)slot_bytes, d_pool + off_qraw, (int64_t)slot_bytes,
                                    cfg.greedy_seed, cfg.greedy_mode, s);
            });
        if (rc) return rc;
    }

    // ---- 2. one slice of sweeps for every resident request -----------------
    ServeTask *h_tasks = reinterpret_cast<ServeTask *>(h_stage + st_tasks);
    // (sequential work of the task, task): each family's tasks are staged
    // longest first, so the slice's long tasks start early and short ones
    // fill the device around them
    using CostTask = std::pair<int64_t, ServeTask>;
    std::vector<CostTask> rows_t, bytes_t, static_t[kStaticMaxD + 1];
    size_t lds_rows = 0, lds_bytes = 0;
    std::vector<int> finished;
    // lanes per chain for this slice: at light load every chain spreads over
    // up to max_lanes_per_chain lanes of the byte-state kernel (lower latency
    // per request); as resident work grows the count halves until the slice
    // fits the wave and LDS budgets, down to each plan's own kernel choice.
    // Every choice gives the same chain trajectories, so it may change from
    // one slice to the next.
    int G = 1;
    for (int g = cfg.max_lanes_per_chain; g > 1; g >>= 1) {
        int64_t waves = 0;
        size_t lds_max = 0;
        for (int s : resident) {
            const Slot &sl = slots[s];
            const int gr = lanes_for(*sl.plan, g);
            waves += (4 * sl.n_rep * gr + kWave - 1) / kWave;
            lds_max = std::max(lds_max, sl.plan->lds_bytes_anneal(gr));
        }
        if (waves <= wave_budget && (size_t)waves * lds_max <= lds_budget) { G = g; break; }
    }
    // work-balanced slice: a request advances sweeps in inverse proportion to
    // the sequential work of one of its sweeps (generators per lane), so every
    // task of the slice carries about the work of sweeps_per_slice sweeps of
    // the costliest resident request
    int64_t ref_cost = 1;
    for (int s : resident) ref_cost = std::max(ref_cost, sweep_cost(*slots[s].plan, G));
    // short slices at light load let arrivals join soon after they come;
    // with more requests resident the slices lengthen (one more
    // sweeps_per_slice per kSliceGrowth requests), so the fixed costs of a
    // slice (admission, host scheduling, the wait for its longest task) stay
    // small against its work
    const int64_t slice_sweeps = (int64_t)cfg.sweeps_per_slice * (1 + (int64_t)resident.size() / kSliceGrowth);
    for (int s : resident) {
        Slot &sl = slots[s];
        const Plan &P = *sl.plan;
        const int64_t share = std::max<int64_t>(1, slice_sweeps * ref_cost / sweep_cost(P, G));
        const int t0 = sl.t, t1 = (int)std::min<int64_t>(P.n_sweeps, t0 + share);
        // a fresh request always gets a first task (it initialises E, E_min
        // and the stored state even for an empty schedule)
        if (t1 > t0 || !sl.started) {
            sl.started = true;
            const bool rows = G == 1 && P.use_rows;
            const int gr = G > 1 ? lanes_for(P, G) : (P.use_rows ? 1 : P.lanes);
            const int C = kWave / gr;
            const size_t lds = rows ? P.lds_bytes_rows() : P.lds_bytes_anneal(gr);
            const int nc = 4 * sl.n_rep;
            uint8_t *base = slot_ptr(s);
            for (int c0 = 0; c0 < nc; c0 += C) {
                ServeTask T{};
                T.plan = P.ddev;
                T.refs = base + off_refs;
                T.states = base + off_states;
                T.e3 = reinterpret_cast<int32_t *>(base + off_e3);
                T.snap = nullptr;
                T.best = nullptr;
                T.cp = base + off_cp;
                T.cpk = reinterpret_cast<uint32_t *>(base + off_cpk);
                T.cpk_words = cpk_words;
                T.cpm = reinterpret_cast<int32_t *>(base + off_cpm);
                T.uid = sl.uid;
                T.n_rep = sl.n_rep;
                T.chain0 = c0;
                T.nchains = std::min(C, nc - c0);
                T.t_begin = t0;
                T.t_end = t1;
                int lg = 0;
                while ((1 << lg) < gr) ++lg;
                T.log_lanes = rows ? 0 : lg;
                T.row_words = rows ? P.row_words : 0;
                const int64_t cost = (int64_t)(t1 - t0) * sweep_cost(P, G);
                if (rows && P.static_d) static_t[serve_class_max(P.static_d)].emplace_back(cost, T);
                else if (rows) { rows_t.emplace_back(cost, T); lds_rows = std::max(lds_rows, lds); }
                else { bytes_t.emplace_back(cost, T); lds_bytes = std::max(lds_bytes, lds); }
            }
            sl.t = t1;
        }
        if (sl.t >= P.n_sweeps) finished.push_back(s);
    }
    // one launch per kernel family: generic packed rows, byte states, and
    // the specialised packed-row kernel of each register class present
    // (largest lattices first)
    std::vector<ServeLaunch> launches;
    size_t nt = 0;
    auto add = [&](std::vector<CostTask> &v, int kind, int d, size_t lds) {
        if (v.empty()) return;
        std::stable_sort(v.begin(), v.end(), [](const CostTask &a, const CostTask &b) { return a.first > b.first; });
        ServeLaunch L{};
        L.tasks = reinterpret_cast<const ServeTask *>(d_stage + st_tasks) + nt;
        L.n = (int32_t)v.size();
        L.kind = kind;
        L.d = d;
        L.lds = lds;
        launches.push_back(L);
        nt += v.size();
    };
    add(rows_t, 0, 0, lds_rows);
    add(bytes_t, 1, 0, lds_bytes);
    static constexpr int kClasses[] = {31, 29, 25, 21, 15, 9};
    for (int c : kClasses) add(static_t[c], 2, c, 0);
    if (nt > max_tasks) { set_error("serving task buffer overflow"); return XZZX_ERANGE; }
    if (nt) {
        size_t at = 0;
        for (const auto *v : {&rows_t, &bytes_t})
            for (const CostTask &ct : *v) h_tasks[at++] = ct.second;
        for (int c : kClasses)
            for (const CostTask &ct : static_t[c]) h_tasks[at++] = ct.second;
        rc = check(hipMemcpyAsync(d_stage + st_tasks, h_tasks, nt * sizeof(ServeTask), hipMemcpyHostToDevice, stream),
                   "stage tasks");
        if (rc) return rc;
        rc = serve_slice(launches.data(), (int)launches.size(), cfg.anneal_seed, stream);
        if (rc) return rc;
        ++slices;
    }

    // ---- 3. finish completed requests -------------------------------------
    const size_t nf = finished.size();
    if (nf) {
        ServeFinish *h_fin = reinterpret_cast<ServeFinish *>(h_stage + st_fin);
        ServeTask *h_rep = reinterpret_cast<ServeTask *>(h_stage + st_fin + align256(slots.size() * sizeof(ServeFinish)));
        size_t lds_rep = 0;
        for (size_t k = 0; k < nf; ++k) {
            const int s = finished[k];
            const Slot &sl = slots[s];
            const Plan &P = *sl.plan;
            uint8_t *base = slot_ptr(s);
            ServeFinish F{};
            F.e3 = reinterpret_cast<const int32_t *>(base + off_e3);
            F.qraw = base + off_qraw;
            F.result = reinterpret_cast<int32_t *>(base + off_res);
            F.recovery = base + off_rec;
            F.out = d_stage + st_out + k * out_stride();
            F.n_rep = sl.n_rep;
            F.nq = P.lat.nq;
            h_fin[k] = F;
            // replay the best chain with every lane of a wavefront on it
            ServeTask T{};
            T.plan = P.ddev;
            T.refs = base + off_refs;
            T.states = base + off_states;
            T.e3 = reinterpret_cast<int32_t *>(base + off_e3);
            T.snap = base + off_rec;
            T.best = reinterpret_cast<const int32_t *>(base + off_res) + 2;
            // from the start state of the sweep range in which the chain's E_min was reached
            T.cp = base + off_cp;
            T.cpk = reinterpret_cast<uint32_t *>(base + off_cpk);
            T.cpk_words = cpk_words;
            T.cpm = reinterpret_cast<int32_t *>(base + off_cpm);
            T.uid = sl.uid;
            T.n_rep = sl.n_rep;
            T.chain0 = 0;
            T.nchains = 1;
            T.t_begin = 0;
            T.t_end = P.n_sweeps;
            T.log_lanes = 6;
            T.row_words = 0;
            h_rep[k] = T;
            lds_rep = std::max(lds_rep, P.lds_bytes_anneal(kWave));
        }
        rc = check(hipMemcpyAsync(d_stage + st_fin, h_stage + st_fin,
                                  align256(slots.size() * sizeof(ServeFinish)) + nf * sizeof(ServeTask),
                                  hipMemcpyHostToDevice, stream), "stage finish");
        if (rc) return rc;
        rc = serve_finish(reinterpret_cast<const ServeFinish *>(d_stage + st_fin),
                          reinterpret_cast<const ServeTask *>(d_stage + st_fin + align256(slots.size() * sizeof(ServeFinish))),
                          (int)nf, lds_rep, cfg.anneal_seed, stream);
        if (rc) return rc;
        // results, gathered on the device as [8 words][recovery max_qubits]
        // per finished request: one copy to the host
        rc = check(hipMemcpyAsync(h_stage + st_out, d_stage + st_out, nf * out_stride(), hipMemcpyDeviceToHost, stream),
                   "results");
        if (rc) return rc;
    }
    rc = check(hipStreamSynchronize(stream), "slice");
    if (rc) return rc;

    // ---- 4. publish ---------------------------------------------------------
    if (nf) {
        const auto now = Clock::now();
        const size_t per = out_stride();
        std::lock_guard<std::mutex> lk(mu);
        for (size_t k = 0; k < nf; ++k) {
            Slot &sl = slots[finished[k]];
            const int32_t *w = reinterpret_cast<const int32_t *>(h_stage + st_out + k * per);
            Done dn;
            dn.e_best = w[0];
            dn.cls = w[1];
            for (int P = 0; P < 4; ++P) dn.e_cls[P] = w[4 + P];
            dn.recovery.assign(h_stage + st_out + k * per + 32, h_stage + st_out + k * per + 32 + sl.plan->lat.nq);
            dn.latency_s = std::chrono::duration<double>(now - sl.submit).count();
            dn.queue_s = std::chrono::duration<double>(sl.admit - sl.submit).count();
            latencies.push_back(dn.latency_s);
            attempts_done += 4.0 * sl.n_rep * sl.plan->n_sweeps * sl.plan->lat.nstab;
            done[sl.ticket] = std::move(dn);
            where.erase(sl.ticket);
            lds_used -= sl.lds;
            sl.busy = false;
            // swap-remove from the resident list, back to the free stack
            const int s = finished[k], at = resident_pos[s], last = resident.back();
            resident[at] = last;
            resident_pos[last] = at;
            resident.pop_back();
            free_slots.push_back(s);
            ++completed;
            last_done = now;
        }
        cv_done.notify_all();
    }
    return XZZX_OK;
}

void xzzx_server::run()
{
    (void)hipSetDevice(device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !pending.empty() || !resident.empty(); });
            if (stop && pending.empty() && resident.empty()) return;
        }
        const int rc = slice();
        if (rc) {
            std::lock_guard<std::mutex> lk(mu);
            error = rc;
            error_msg = xzzx_last_error();
            stop = true;
            cv_done.notify_all();
            return;
        }
    }
}

extern "C" {

int xzzx_server_create(const xzzx_server_cfg *cfg, xzzx_server **out)
{
    if (!cfg || !out) { set_error("NULL argument"); return XZZX_EINVAL; }
    *out = nullptr;
    if (cfg->max_slots < 1 || cfg->max_rep < 1 || cfg->max_qubits < 9 || cfg->max_qubits > 2047 ||
        cfg->sweeps_per_slice < 1 || cfg->max_pending < 1 || cfg->lds_budget_bytes < 0 ||
        cfg->max_lanes_per_chain < 0 || cfg->max_lanes_per_chain > kWave ||
        (cfg->max_lanes_per_chain & (cfg->max_lanes_per_chain - 1)) != 0 || cfg->max_waves < 0 ||
        (cfg->greedy_mode != XZZX_GREEDY_RANDOM && cfg->greedy_mode != XZZX_GREEDY_SAME &&
         cfg->greedy_mode != XZZX_GREEDY_BOUNDARY)) {
        set_error("bad server configuration");
        return XZZX_EINVAL;
    }
    auto *S = new (std::nothrow) xzzx_server();
    if (!S) { set_error("out of host memory"); return XZZX_ENOMEM; }
    S->cfg = *cfg;
    int rc = check(hipGetDevice(&S->device), "hipGetDevice");
    int cus = 0, lds_cu = 0;
    if (!rc) rc = check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, S->device), "CU count");
    if (!rc && hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, S->device) != hipSuccess)
        lds_cu = 160 * 1024;
    if (lds_cu <= 0) lds_cu = 160 * 1024;
    // default: four times the device's LDS, so that under load a slice holds
    // more tasks than the CUs run at once and the waves whose short tasks end
    // early (small lattices) take queued ones instead of idling
    S->lds_budget = cfg->lds_budget_bytes ? (size_t)cfg->lds_budget_bytes : 4 * (size_t)cus * (size_t)lds_cu;
    S->wave_budget = cfg->max_waves ? cfg->max_waves : 32 * (int64_t)cus;
    if (!S->cfg.max_lanes_per_chain) S->cfg.max_lanes_per_chain = kWave;
    const size_t nq = (size_t)cfg->max_qubits, R = (size_t)cfg->max_rep;
    S->max_nstab = cfg->max_qubits;   // n_stabs < n_qubits for both layouts
    S->off_refs = 0;
    S->off_states = align256(R * nq);
    S->off_e3 = S->off_states + align256(4 * R * nq);
    S->off_qraw = S->off_e3 + align256(3 * 4 * R * 4);
    S->off_res = S->off_qraw + align256(R);
    S->off_rec = S->off_res + 256;
    S->off_cp = S->off_rec + align256(nq);
    // packed rows of the largest rotated lattice that fits max_qubits
    int dmax = 1;
    while ((size_t)(dmax + 1) * (dmax + 1) <= nq) ++dmax;
    S->cpk_words = dmax * ((2 * (dmax + 1) + 31) / 32);
    S->off_cpk = S->off_cp + align256(2 * 4 * R * nq);
    S->off_cpm = S->off_cpk + align256(2 * 4 * R * (size_t)S->cpk_words * 4);
    S->slot_bytes = S->off_cpm + align256(4 * R * 4);
    const size_t ns = (size_t)cfg->max_slots;
    S->max_tasks = ns * 4 * R;
    S->st_syn = 0;
    S->st_uid = align256(ns * (size_t)S->max_nstab);
    S->st_map = S->st_uid + align256(ns * 4);
    S->st_tasks = S->st_map + align256(ns * 4);
    S->st_fin = S->st_tasks + align256(S->max_tasks * sizeof(ServeTask));
    S->st_out = S->st_fin + align256(ns * sizeof(ServeFinish)) + align256(ns * sizeof(ServeTask));
    S->stage_bytes = S->st_out + align256(ns * S->out_stride());
    if (!rc) rc = check(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking), "stream");
    if (!rc && hipMalloc(&S->d_pool, S->slot_bytes * ns) != hipSuccess) { S->d_pool = nullptr; set_error("slot pool allocation"); rc = XZZX_ENOMEM; }
    if (!rc && hipMalloc(&S->d_stage, S->stage_bytes) != hipSuccess) { S->d_stage = nullptr; set_error("staging allocation"); rc = XZZX_ENOMEM; }
    if (!rc && hipHostMalloc(&S->h_stage, S->stage_bytes, hipHostMallocDefault) != hipSuccess) { S->h_stage = nullptr; set_error("pinned staging"); rc = XZZX_ENOMEM; }
    if (rc) {
        if (S->h_stage) (void)hipHostFree(S->h_stage);
        if (S->d_stage) (void)hipFree(S->d_stage);
        if (S->d_pool) (void)hipFree(S->d_pool);
        if (S->stream) (void)hipStreamDestroy(S->stream);
        delete S;
        return rc;
    }
    S->slots.resize(ns);
    S->resident_pos.assign(ns, -1);
    S->resident.reserve(ns);
    for (int i = ns - 1; i >= 0; --i) S->free_slots.push_back(i);
    S->worker = std::thread([S] { S->run(); });
    *out = S;
    return XZZX_OK;
}

// a request the server can hold, or the error it gets
static int check_request(const xzzx_server *srv, const xzzx_request *req)
{
    if (!req || !req->plan || !req->syndrome) { set_error("NULL argument"); return XZZX_EINVAL; }
    const Plan &P = req->plan->P;
    if (P.order != XZZX_ORDER_COLOUR || P.ladder_k) {
        set_error("the serving loop runs annealing plans with colour sweeps only");
        return XZZX_EINVAL;
    }
    if (req->n_rep < 1 || req->n_rep > srv->cfg.max_rep || P.lat.nq > srv->cfg.max_qubits || P.device != srv->device) {
        set_error("request does not fit the server's slots (n_rep, qubits or device)");
        return XZZX_EINVAL;
    }
    if (request_lds(P, req->n_rep) > srv->lds_budget) { set_error("request needs more LDS than the budget"); return XZZX_EINVAL; }
    return XZZX_OK;
}

// queue requests [0, n) in order under one lock; *n_done of them queued
static int submit_requests(xzzx_server *srv, const xzzx_request *reqs, int n, uint64_t *tickets, int *n_done)
{
    *n_done = 0;
    std::vector<Pending> batch((size_t)n);
    const auto now = Clock::now();
    int rc = XZZX_OK, ok = 0;
    for (; ok < n; ++ok) {
        rc = check_request(srv, &reqs[ok]);
        if (rc) break;
        Pending &p = batch[(size_t)ok];
        p.plan = reqs[ok].plan;
        p.syn.assign(reqs[ok].syndrome, reqs[ok].syndrome + reqs[ok].plan->P.lat.nstab);
        p.uid = reqs[ok].uid;
        p.n_rep = reqs[ok].n_rep;
        p.submit = now;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->error) { set_error(srv->error_msg); return srv->error; }
    for (int i = 0; i < ok; ++i) {
        if ((int)srv->pending.size() >= srv->cfg.max_pending) {
            ++srv->rejected;
            set_error("server queue full");
            rc = XZZX_EAGAIN;
            break;
        }
        Pending &p = batch[(size_t)i];
        p.ticket = srv->next_ticket++;
        tickets[i] = p.ticket;
        srv->where[p.ticket] = 0;
        srv->pending.push_back(std::move(p));
        ++srv->submitted;
        ++*n_done;
    }
    if (*n_done) srv->cv_work.notify_one();
    return rc;
}

int xzzx_server_submit(xzzx_server *srv, const xzzx_request *req, uint64_t *ticket)
{
    if (!srv || !req || !ticket) { set_error("NULL argument"); return XZZX_EINVAL; }
    int done = 0;
    return submit_requests(srv, req, 1, ticket, &done);
}

int xzzx_server_submit_many(xzzx_server *srv, const xzzx_request *reqs, int n, uint64_t *tickets, int *n_done)
{
    if (!srv || !n_done) { set_error("NULL argument"); return XZZX_EINVAL; }
    *n_done = 0;
    if (n < 0 || (n > 0 && (!reqs || !tickets))) { set_error("bad request array"); return XZZX_EINVAL; }
    if (n == 0) return XZZX_OK;
    return submit_requests(srv, reqs, n, tickets, n_done);
}

int xzzx_server_poll(xzzx_server *srv, uint64_t ticket, xzzx_result *out)
{
    if (!srv || !out) { set_error("NULL argument"); return XZZX_EINVAL; }
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->done.find(ticket);
    if (it == srv->done.end()) {
        if (srv->error) { set_error(srv->error_msg); return srv->error; }
        if (srv->where.count(ticket)) return XZZX_ENOTREADY;
        set_error("unknown ticket");
        return XZZX_EINVAL;
    }
    const Done &d = it->second;
    out->e_best = d.e_best;
    out->cls = d.cls;
    for (int P = 0; P < 4; ++P) out->e_cls[P] = d.e_cls[P];
    if (out->recovery) std::memcpy(out->recovery, d.recovery.data(), d.recovery.size());
    out->latency_s = d.latency_s;
    out->queue_s = d.queue_s;
    srv->done.erase(it);
    return XZZX_OK;
}

int xzzx_server_drain(xzzx_server *srv)
{
    if (!srv) { set_error("NULL argument"); return XZZX_EINVAL; }
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->error != XZZX_OK || srv->where.empty(); });
    if (srv->error) { set_error(srv->error_msg); return srv->error; }
    return XZZX_OK;
}

int xzzx_server_stats(xzzx_server *srv, xzzx_serve_stats *out)
{
    if (!srv || !out) { set_error("NULL argument"); return XZZX_EINVAL; }
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = xzzx_serve_stats{};
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->rejected = srv->rejected;
    out->slices = srv->slices;
    if (!srv->latencies.empty()) {
        std::vector<double> v = srv->latencies;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            const size_t i = (size_t)std::min<double>((double)v.size() - 1, std::max(0.0, std::ceil(q * v.size()) - 1));
            return v[i];
        };
        out->p50_latency_s = pct(0.50);
        out->p99_latency_s = pct(0.99);
        double sum = 0;
        for (double x : v) sum += x;
        out->mean_latency_s = sum / v.size();
        out->busy_s = std::chrono::duration<double>(srv->last_done - srv->first_admit).count();
        if (out->busy_s > 0) {
            out->decodes_per_s = srv->completed / out->busy_s;
            out->attempts_per_s = srv->attempts_done / out->busy_s;
        }
    }
    return XZZX_OK;
}

void xzzx_server_destroy(xzzx_server *srv)
{
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    (void)hipStreamSynchronize(srv->stream);
    if (srv->h_stage) (void)hipHostFree(srv->h_stage);
    if (srv->d_stage) (void)hipFree(srv->d_stage);
    if (srv->d_pool) (void)hipFree(srv->d_pool);
    if (srv->stream) (void)hipStreamDestroy(srv->stream);
    delete srv;
}

}  // extern "C"
