// gfx950 kernels of the XZZX simulated-annealing decoder and the device-side
// entry points of the C ABI.
//
//   k_syndrome  Eq. (2): syndrome of a batch of configurations.
//   k_greedy    Algs. 5-6: greedy matching per (syndrome, replica), both
//               decoding-graph colours, paths XOR-ed into an LDS configuration.
//   k_qcls      Alg. 7: class Q_r of each reference relative to replica 0.
//   k_anneal    Algs. 2-3: the hot loop.  Persistent wavefronts pull tasks of
//               C = 64/G chains from an atomic queue spanning every syndrome
//               group of the launch (uneven distances allowed).  Each chain's
//               byte-per-qubit state lives in LDS, interleaved across the C
//               chains of the wavefront; the G lanes of a chain split the
//               generators of one colour class (qubit-disjoint, so they update
//               concurrently).  Replay mode re-runs the best chain of each
//               syndrome up to the phase of its minimum and stores that state.
//   k_reduce    Eqs. (18)-(21): per-coset minima, P*, best chain.
#include <hip/hip_runtime.h>

#include <utility>

#include <algorithm>
#include <cstring>
#include <vector>

#include "xzzx_internal.h"

namespace xzzx {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// by the Philox multipliers, high/low halves crossed with the other words and
// the round key; the key advances by the two Weyl increments.
// ---------------------------------------------------------------------------
// Three-input XOR as one gfx950 v_bitop3_b32 (truth table 0x96 = odd parity).
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t key)
{
    return __builtin_amdgcn_bitop3_b32(a, b, key, 0x96);
}

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t p0 = (uint64_t)c.x * 0xD2511F53u;
        const uint64_t p1 = (uint64_t)c.z * 0xCD9E8D57u;
        c = make_uint4(xor3_key((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1,
                       xor3_key((uint32_t)(p0 >> 32), c.w, k1), (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ void wave_lds_fence()
{
    // Orders this wavefront's LDS traffic across a phase boundary: all lanes
    // see the stores of the previous phase before any load of the next one.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int32_t weight_of(const int32_t W[4], uint32_t code)
{
    return code == 0 ? 0 : code == 1 ? W[1] : code == 2 ? W[2] : W[3];
}

// Sum over the G lanes of one chain (lanes c*G .. c*G+G-1 of the wavefront).
template <int LOGG>
__device__ __forceinline__ int32_t chain_sum(int32_t v)
{
#pragma unroll
    for (int s = 1; s < (1 << LOGG); s <<= 1) v += __shfl_xor(v, s, kWave);
    return v;
}

// ---------------------------------------------------------------------------
// Syndrome, Eq. (2): s_f = 1 iff the configuration anticommutes with G_f.
// Slots 0 and 3 carry X (detect a Z component), slots 1 and 2 carry Z (detect
// an X component).
// ---------------------------------------------------------------------------
__global__ void k_syndrome(const PlanDev *__restrict__ pl, const uint8_t *__restrict__ cfg,
                           int64_t n, uint8_t *__restrict__ syn)
{
    const int nstab = pl->nstab, nq = pl->nq;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * nstab) return;
    const int64_t s = idx / nstab;
    const int f = (int)(idx - s * nstab);
    const Desc d = pl->face_desc[f];
    const int q[4] = {(int)(d.x & 0xFFFF), (int)(d.x >> 16), (int)(d.y & 0xFFFF), (int)((d.y >> 16) & 0x7FF)};
    const uint8_t *c = cfg + s * nq;
    uint32_t bit = 0;
    if (q[0] < nq) bit ^= c[q[0]] & 1;
    if (q[1] < nq) bit ^= (c[q[1]] >> 1) & 1;
    if (q[2] < nq) bit ^= (c[q[2]] >> 1) & 1;
    if (q[3] < nq) bit ^= c[q[3]] & 1;
    syn[idx] = (uint8_t)bit;
}

// ---------------------------------------------------------------------------
// Greedy matching (Algs. 5-6) -- one wavefront per (syndrome, replica).
//
// The sequential rule "take the free pair of least (weight, key, pair id)"
// is evaluated as repeated mutual-best elimination: every free defect finds
// its least free partner, and pairs that are each other's least are matched.
// Under a strict total order the pair taken first by the sequential scan is
// always mutual-best, and removing matched defects never changes the order of
// the rest, so both procedures produce the same matching.  Paths follow the
// canonical tight-edge walk (smallest edge id) and are XOR-ed into the
// configuration with LDS atomics (paths may overlap).
// ---------------------------------------------------------------------------
struct GreedyArgs {
    const PlanDev *plan;
    const uint8_t *syn;
    const uint32_t *uid;
    uint8_t *refs;
    uint8_t *qraw;
    int64_t syn_stride;        // bytes between syndromes
    const int32_t *slot_map;   // optional: syndrome s writes to slot slot_map[s]
    int64_t refs_stride;       // bytes between slots (with slot_map)
    int64_t qraw_stride;
    int64_t n_syn;
    int n_rep;
    int mode;
    uint32_t seed_lo, seed_hi;
    int max_nodes;
};

__device__ __forceinline__ void xor_edge(uint32_t *cfgw, int eid)
{
    const int q = eid >> 1;
    const uint32_t code = (eid & 1) ? 2u : 1u;
    atomicXor(&cfgw[q >> 2], code << (8 * (q & 3)));
}

__device__ void walk_interior(const PlanDev *pl, int g, int u, int v, uint32_t *cfgw)
{
    const int n = pl->ncol[g];
    const int32_t *du = pl->dint[g] + (size_t)u * n;
    const int4 *adj = pl->adj[g];
    int x = v;
    for (int step = 0; step < n && x != u; ++step) {
        const int32_t dx = du[x];
        int nxt = -1;
        for (int s = 0; s < 4; ++s) {
            const int4 e = adj[4 * x + s];
            if (e.x < 0 || e.y < 0) continue;
            if (du[e.y] + e.z == dx) { xor_edge(cfgw, e.x); nxt = e.y; break; }
        }
        if (nxt < 0) return;
        x = nxt;
    }
}

__device__ void walk_boundary(const PlanDev *pl, int g, int u, uint32_t *cfgw)
{
    const int n = pl->ncol[g];
    const int32_t *db = pl->db[g];
    const int4 *adj = pl->adj[g];
    int x = u;
    for (int step = 0; step <= n; ++step) {
        const int32_t dx = db[x];
        int nxt = -1;
        for (int s = 0; s < 4; ++s) {
            const int4 e = adj[4 * x + s];
            if (e.x < 0) continue;
            if (e.y < 0) {
                if (e.z == dx) { xor_edge(cfgw, e.x); return; }
            } else if (db[e.y] + e.z == dx) {
                xor_edge(cfgw, e.x);
                nxt = e.y;
                break;
            }
        }
        if (nxt < 0) return;
        x = nxt;
    }
}

__global__ __launch_bounds__(kWave) void k_greedy(GreedyArgs A)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const PlanDev *pl = A.plan;
    const int lane = threadIdx.x;
    const int nq = pl->nq;
    const int64_t sr = blockIdx.x;
    const int64_t s = sr / A.n_rep;
    const uint32_t r = (uint32_t)(sr - s * A.n_rep);
    const uint32_t uid = A.uid[s];
    const int nwords = (nq + 3) / 4;
    uint32_t *cfgw = reinterpret_cast<uint32_t *>(smem);
    int32_t *D = reinterpret_cast<int32_t *>(smem + 4 * nwords);
    int32_t *best = D + A.max_nodes + 1;
    int32_t *pairs = best + A.max_nodes + 1;
    uint8_t *freef = reinterpret_cast<uint8_t *>(pairs + A.max_nodes + 1);
    __shared__ int s_count;

    for (int i = lane; i < nwords; i += kWave) cfgw[i] = 0;
    const uint8_t *sy = A.syn + s * A.syn_stride;
    for (int g = 0; g < 2; ++g) {
        const int n = pl->ncol[g];
        const int32_t *cf = pl->col_face[g];
        const int32_t *dint = pl->dint[g];
        const int32_t *db = pl->db[g];
        // defects of this colour, ascending node index
        int nd = 0;
        for (int base = 0; base < n; base += kWave) {
            const int v = base + lane;
            const bool flag = v < n && sy[cf[v]];
            const uint64_t mask = __ballot(flag);
            const int pos = nd + __popcll(mask & ((1ull << lane) - 1ull));
            if (flag) D[pos] = v;
            nd += __popcll(mask);
        }
        __syncthreads();
        if (A.mode == XZZX_GREEDY_BOUNDARY) {
            for (int i = lane; i < nd; i += kWave) walk_boundary(pl, g, D[i], cfgw);
            __syncthreads();
            continue;
        }
        const int na = nd + (nd & 1);   // odd count: the virtual boundary joins as node nd
        for (int i = lane; i < na; i += kWave) freef[i] = 1;
        if (lane == 0) s_count = 0;
        __syncthreads();
        int nfree = na;
        const bool randomized = A.mode == XZZX_GREEDY_RANDOM;
        // every round matches at least the least free pair, so na/2 rounds suffice
        for (int round = 0; nfree > 0 && round <= na / 2; ++round) {
            for (int i = lane; i < na; i += kWave) {
                if (!freef[i]) continue;
                uint32_t bw = 0xFFFFFFFFu, bk = 0xFFFFFFFFu, bid = 0xFFFFFFFFu;
                int bj = -1;
                for (int j = 0; j < na; ++j) {
                    if (j == i || !freef[j]) continue;
                    const int lo = min(i, j), hi = max(i, j);
                    uint32_t w;
                    if (hi == nd) {
                        w = (uint32_t)db[D[lo]];
                    } else {
                        const int u = D[lo], v = D[hi];
                        w = (uint32_t)min(dint[(size_t)u * n + v], db[u] + db[v]);
                    }
                    const uint32_t id = (uint32_t)(lo * na + hi);
                    if (w > bw) continue;
                    const uint32_t key = randomized
                        ? philox4x32_10(make_uint4(uid, r, 0x100u + (uint32_t)g, id), A.seed_lo, A.seed_hi).x
                        : 0u;
                    if (w < bw || key < bk || (key == bk && id < bid)) { bw = w; bk = key; bid = id; bj = j; }
                }
                best[i] = bj;
            }
            __syncthreads();
            for (int i = lane; i < na; i += kWave) {
                if (!freef[i]) continue;
                const int j = best[i];
                if (j > i && best[j] == i) {
                    const int p = atomicAdd(&s_count, 1);
                    pairs[p] = i | (j << 16);
                }
            }
            __syncthreads();
            const int np = s_count;
            for (int p = lane; p < np; p += kWave) {
                freef[pairs[p] & 0xFFFF] = 0;
                freef[pairs[p] >> 16] = 0;
            }
            __syncthreads();
            nfree = na - 2 * np;
        }
        const int np = s_count;
        for (int p = lane; p < np; p += kWave) {
            const int i = pairs[p] & 0xFFFF, j = pairs[p] >> 16;
            if (j == nd) {
                walk_boundary(pl, g, D[i], cfgw);
            } else {
                const int u = D[i], v = D[j];
                if (dint[(size_t)u * n + v] <= db[u] + db[v]) {
                    walk_interior(pl, g, u, v, cfgw);
                } else {
                    walk_boundary(pl, g, u, cfgw);
                    walk_boundary(pl, g, v, cfgw);
                }
            }
        }
        __syncthreads();
    }
    // write the reference and its symplectic products with L_Z and L_X
    uint8_t *out = A.slot_map ? A.refs + A.slot_map[s] * A.refs_stride + (size_t)r * nq : A.refs + (size_t)sr * nq;
    uint8_t *qraw_out = A.slot_map ? A.qraw + A.slot_map[s] * A.qraw_stride + r : A.qraw + sr;
    const uint8_t *cb = reinterpret_cast<const uint8_t *>(cfgw);
    uint32_t vz = 0, vx = 0;
    for (int q = lane; q < nq; q += kWave) {
        const uint32_t c = cb[q];
        out[q] = (uint8_t)c;
        const uint32_t z = pl->lz[q], x = pl->lx[q];
        vz ^= (((c >> 1) & z) ^ (c & (z >> 1))) & 1;
        vx ^= (((c >> 1) & x) ^ (c & (x >> 1))) & 1;
    }
    const int az = __popcll(__ballot(vz)) & 1;
    const int ax = __popcll(__ballot(vx)) & 1;
    if (lane == 0) *qraw_out = (uint8_t)(az | (ax << 1));
}

// Pauli class index (I=0, X=1, Y=2, Z=3) <-> (x, z) bits, and products.
__device__ __forceinline__ int cls_from_bits(int x, int z) { return x ? (z ? 2 : 1) : (z ? 3 : 0); }
__device__ __forceinline__ int cls_x(int c) { return (c == 1) | (c == 2); }
__device__ __forceinline__ int cls_z(int c) { return (c == 2) | (c == 3); }
__device__ __forceinline__ int cls_mul(int a, int b) { return cls_from_bits(cls_x(a) ^ cls_x(b), cls_z(a) ^ cls_z(b)); }

// Class of R_r relative to R_0 from the symplectic products with L_Z (bit 0:
// an X-type logical anticommutes with L_Z) and L_X (bit 1).  One thread per
// syndrome reads replica 0 first, so qcls may alias qraw.
__global__ void k_qcls(const uint8_t *qraw, int64_t n_syn, int n_rep, uint8_t *qcls)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_syn) return;
    const int r0 = qraw[s * n_rep] & 3;
    for (int r = 0; r < n_rep; ++r) {
        const int v = (qraw[s * n_rep + r] & 3) ^ r0;
        qcls[s * n_rep + r] = (uint8_t)cls_from_bits(v & 1, v >> 1);
    }
}

// ---------------------------------------------------------------------------
// Annealing (Algs. 2-3).
//
// Both annealing kernels run a chain from a per-lane ChainJob: start at the
// replica reference R_r times the coset's logical L_P' (or resume from a
// saved state with its E, E_min and phase of the minimum), run sweeps
// [t_begin, t_end) of the plan's schedule, then store E, E_min, the phase of
// E_min and optionally the state.  Replay jobs stop at the phase of the
// chain's minimum and store that state (the recovery).  A task is a set of
// chains sharing a plan and a sweep range; the batch launch builds its tasks
// from syndrome groups, the serving loop from its resident requests.
// ---------------------------------------------------------------------------
struct ChainJob {
    const uint8_t *src;    // start: reference R_r; resume: saved state
    int32_t *emin, *stop, *efin;   // result word arrays (wave-uniform bases), entry ci
    uint8_t *states;       // end-of-range states (wave-uniform base, stride nq), entry ci; nullable
    uint8_t *snap;         // replay: destination of the state at `target`
    int64_t ci;            // this chain's entry in the result arrays
    uint32_t uid;          // syndrome id (RNG counter word 0)
    uint32_t cc;           // chain index in its syndrome (RNG counter word 1)
    int32_t lp;            // coset logical applied at start (0..3)
    int32_t target;        // replay: phase whose state is stored (-1 = none)
    bool active, resume;
    // checkpoints of the specialised packed-row kernel (word-major rows of
    // rows 1..d, plane stride cp_stride chains)
    uint32_t *cp_out;      // anneal: checkpoint planes to write (nullable), base of checkpoint 0
    const uint32_t *cp_in; // replay: packed rows to start from instead of src (nullable)
    int64_t cp_stride;     // chains per word plane
    int32_t t0;            // first sweep to run (replay from a checkpoint)
};

struct GroupArgs {
    const PlanDev *plan;
    const uint32_t *uid;
    const uint8_t *refs;          // [n_syn][n_rep][nq]
    int32_t *emin, *stop, *efin;  // [n_syn][4 n_rep]
    uint8_t *final;               // optional [n_syn][4 n_rep][nq]
    const int32_t *best_chain;    // replay: [n_syn]
    uint8_t *recovery;            // replay: [n_syn][nq]
    int64_t unit_offset;          // first unit (chain or syndrome) of this launch
    int64_t n_units;              // units handled by this launch
    int64_t task_begin;           // first task index of this group
    int n_rep;
    int log_lanes;
    int row_words;                // packed-row kernel: words per row (1 or 2)
    uint32_t *cp_rows;            // specialised packed-row kernel: checkpoints [n_cp][d][n_chains]
    int64_t n_chains;             // chains of the whole group
    int cp_every;                 // sweeps between checkpoints (0 = none)
};

struct AnnealArgs {
    GroupArgs g[kMaxGroups];
    int n_groups;
    uint32_t n_tasks;
    uint32_t *counter;
    uint32_t seed_lo, seed_hi;
};

// Batch job of the chain (or, in replay, syndrome) `unit` of group G.
__device__ __forceinline__ ChainJob batch_job(const GroupArgs &G, int64_t unit, bool replay)
{
    ChainJob j;
    const int nc = 4 * G.n_rep;
    j.active = unit < G.n_units;
    const int64_t u_abs = G.unit_offset + (j.active ? unit : 0);
    int64_t s, ci;
    if (replay) {
        s = u_abs;
        j.cc = (uint32_t)G.best_chain[s];
        ci = s * nc + j.cc;
        j.target = G.stop[ci];
        j.snap = G.recovery + (size_t)s * G.plan->nq;
    } else {
        s = u_abs / nc;
        ci = u_abs;
        j.cc = (uint32_t)(u_abs - s * nc);
        j.target = -1;
        j.snap = nullptr;
    }
    const int r = (int)(j.cc >> 2);
    j.lp = (int)(j.cc & 3);
    j.uid = G.uid[s];
    j.src = G.refs + ((size_t)s * G.n_rep + r) * G.plan->nq;
    j.resume = false;
    j.ci = ci;
    j.emin = G.emin;
    j.stop = G.stop;
    j.efin = G.efin;
    j.states = replay ? nullptr : G.final;
    j.cp_out = replay ? nullptr : G.cp_rows;
    j.cp_in = nullptr;
    j.cp_stride = G.n_chains;
    j.t0 = 0;
    if (replay && G.cp_rows && j.target > 0) {
        // start from the last checkpoint at or before the sweep of the target phase
        const int t_target = (j.target - 1) >> 2;
        const int n_cp = t_target / G.cp_every;
        if (n_cp > 0) {
            j.cp_in = G.cp_rows + (int64_t)(n_cp - 1) * G.plan->d * G.n_chains + ci;
            j.t0 = n_cp * G.cp_every;
        }
    }
    return j;
}

struct LdsLayout {
    uint32_t desc, lut, et, state;
};

__device__ __forceinline__ LdsLayout lds_layout(int M, int ntypes, int nranks)
{
    LdsLayout o;
    o.desc = 0;
    o.lut = 8u * 4u * (uint32_t)M;
    o.et = (o.lut + 256u * (uint32_t)ntypes + 7u) & ~7u;
    o.state = (o.et + 8u * (uint32_t)nranks + 15u) & ~15u;
    return o;
}

// Byte-state core: C = 64/G chains per wavefront, chain c on lanes c*G..c*G+G-1;
// the G lanes of a chain split the generators of each colour class.
template <int LOGG, bool REPLAY>
__device__ void bytes_core(const PlanDev *pl, const ChainJob &J, int t_begin, int t_end, uint32_t seed_lo,
                           uint32_t seed_hi, uint8_t *smem)
{
    constexpr int LOGC = 6 - LOGG;
    const int lane = threadIdx.x;
    const int c = lane >> LOGG;          // chain slot in this wavefront
    const int gl = lane & ((1 << LOGG) - 1);
    const int nq = pl->nq, M = pl->M, nblk = pl->nblk, nranks = pl->nranks;
    const uint32_t kneg = (uint32_t)pl->kneg;
    int32_t W[4];
    W[0] = pl->W[0]; W[1] = pl->W[1]; W[2] = pl->W[2]; W[3] = pl->W[3];
    const LdsLayout lo = lds_layout(M, pl->ntypes, nranks);
    const uint2 *desc_s = reinterpret_cast<const uint2 *>(smem + lo.desc);
    const uint8_t *lut_s = smem + lo.lut;
    int2 *et_s = reinterpret_cast<int2 *>(smem + lo.et);
    uint8_t *st = smem + lo.state;
    const uint32_t uid = J.uid, cc = J.cc;

    // initial state, interleaved: qubit q of slot c at q*C + c
    const bool use_x = (J.lp == 1 || J.lp == 2), use_z = (J.lp == 2 || J.lp == 3);
    int32_t part = 0;
    const int dd = pl->d;
    for (int q = gl; q < nq; q += (1 << LOGG)) {
        uint32_t v;
        if (J.cp_in) {
            // checkpoint rows (rotated lattice): row y of qubit q, 2 bits at column x + 1
            const int y = q / dd, x = q - y * dd;
            v = J.active ? (J.cp_in[(int64_t)y * J.cp_stride] >> (2 * (x + 1))) & 3u : 0u;
        } else {
            v = J.active ? (J.src[q] & 3u) : 0u;
            if (!J.resume) {
                if (use_x) v ^= pl->lx[q];
                if (use_z) v ^= pl->lz[q];
            }
        }
        st[(q << LOGC) + c] = (uint8_t)v;
        part += weight_of(W, v);
    }
    if (gl == 0) st[(nq << LOGC) + c] = 0;
    int32_t E = chain_sum<LOGG>(part);
    int32_t Emin = E, stop = 0;
    if (J.resume && J.active) {
        E = J.efin[J.ci];
        Emin = J.emin[J.ci];
        stop = J.stop[J.ci];
    }
    wave_lds_fence();

    auto save_state = [&](uint8_t *dst) {
        for (int q = gl; q < nq; q += (1 << LOGG)) dst[q] = st[(q << LOGC) + c];
    };
    int32_t last_phase = 4 * t_end;
    if (REPLAY) {
        if (J.active && J.target == 0) save_state(J.snap);
        int32_t tmax = J.active ? J.target : 0;
#pragma unroll
        for (int sh = 1; sh < kWave; sh <<= 1) tmax = max(tmax, __shfl_xor(tmax, sh, kWave));
        last_phase = tmax;
    }

    for (int t = t_begin; t < t_end && 4 * t < last_phase; ++t) {
        for (int i = lane; i < nranks; i += kWave) et_s[i].y = (int)pl->thr[(size_t)t * nranks + i];
        wave_lds_fence();
        for (int k = 0; k < 4; ++k) {
            const uint2 *dk = desc_s + k * M;
            int32_t acc_de = 0;
            for (int b = gl; b < nblk; b += (1 << LOGG)) {
                const uint4 rnd = philox4x32_10(make_uint4(uid, cc, 4u * (uint32_t)t + (uint32_t)k, (uint32_t)b),
                                                seed_lo, seed_hi);
                const uint32_t uw[4] = {rnd.x, rnd.y, rnd.z, rnd.w};
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const int m = 4 * b + w;
                    if (m >= M) break;
                    const uint2 d = dk[m];
                    const uint32_t a0 = ((d.x & 0xFFFFu) << LOGC) + c;
                    const uint32_t a1 = ((d.x >> 16) << LOGC) + c;
                    const uint32_t a2 = ((d.y & 0xFFFFu) << LOGC) + c;
                    const uint32_t a3 = (((d.y >> 16) & 0x7FFu) << LOGC) + c;
                    const uint32_t c0 = st[a0], c1 = st[a1], c2 = st[a2], c3 = st[a3];
                    const uint32_t pat = c0 | (c1 << 2) | (c2 << 4) | (c3 << 6);
                    const uint32_t rank = lut_s[((d.y >> 27) << 8) | pat];
                    const int2 et = et_s[rank];
                    if (rank < kneg || uw[w] < (uint32_t)et.y) {
                        st[a0] = (uint8_t)(c0 ^ 2u);
                        st[a1] = (uint8_t)(c1 ^ 1u);
                        st[a2] = (uint8_t)(c2 ^ 1u);
                        st[a3] = (uint8_t)(c3 ^ 2u);
                        acc_de += et.x;
                    }
                }
            }
            wave_lds_fence();
            E += chain_sum<LOGG>(acc_de);
            const int32_t phase = 4 * t + k + 1;
            if (E < Emin) { Emin = E; stop = phase; }
            if (REPLAY && J.active && phase == J.target) save_state(J.snap);
        }
    }
    if (!REPLAY && J.active) {
        if (gl == 0) {
            J.emin[J.ci] = Emin;
            J.stop[J.ci] = stop;
            J.efin[J.ci] = E;
        }
        if (J.states) save_state(J.states + (size_t)J.ci * nq);
    }
    wave_lds_fence();
}

// ---------------------------------------------------------------------------
// Packed-row core (rotated lattices, d <= 29): one chain per lane.  The padded
// grid (columns and rows -1..d) is stored as 2-bit codes, each lattice row in
// NW 32-bit words; word w of row Y of the chain in lane l sits at
// rows_s[(Y*NW + w)*64 + l], so a wavefront's row accesses are 64 consecutive
// dwords.  The generators of a colour class are visited in rank order; a
// generator at cell (i,j) covers the 4-bit nibble at bit 2(i+1) of rows j+1
// (slots X_left, Z_up) and j+2 (slots Z_down, X_right).  The two rows are held
// in registers while the class visits that row, so LDS traffic per move is the
// two table lookups.  Generator tables are uniform across the wavefront and
// read through the scalar cache.
// ---------------------------------------------------------------------------
typedef const __attribute__((address_space(4))) uint32_t const_u32;

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

struct RowsLds {
    uint32_t lut, et, rows;
};

__device__ __forceinline__ RowsLds rows_layout(int ntypes, int nranks)
{
    RowsLds o;
    o.lut = 0;
    o.et = (256u * (uint32_t)ntypes + 7u) & ~7u;
    o.rows = (o.et + 8u * (uint32_t)nranks + 15u) & ~15u;
    return o;
}

template <int NW>
__device__ __forceinline__ uint32_t row_nibble(const uint32_t (&r)[NW], uint32_t bo)
{
    if (NW == 1) return __builtin_amdgcn_ubfe(r[0], bo, 4);
    if (bo < 32) return __builtin_amdgcn_alignbit(r[NW > 1 ? 1 : 0], r[0], bo) & 0xFu;
    return __builtin_amdgcn_ubfe(r[NW > 1 ? 1 : 0], bo - 32, 4);
}

template <int NW>
__device__ __forceinline__ void row_flip(uint32_t (&r)[NW], uint32_t bo, uint32_t mask)
{
    if (NW == 1) {
        r[0] ^= mask << bo;
        return;
    }
    if (bo < 32) {
        r[0] ^= mask << bo;
        if (bo > 28) r[NW > 1 ? 1 : 0] ^= mask >> (32 - bo);
    } else {
        r[NW > 1 ? 1 : 0] ^= mask << (bo - 32);
    }
}

// r ^= (mask << bo) & sel as one v_bitop3 per word (truth table 0x6A:
// c ^ (a & b) with a = shifted mask, b = sel, c = r).
__device__ __forceinline__ uint32_t xor_and(uint32_t r, uint32_t mask, uint32_t sel)
{
    return __builtin_amdgcn_bitop3_b32(mask, sel, r, 0x6A);
}

template <int NW>
__device__ __forceinline__ void row_flip_sel(uint32_t (&r)[NW], uint32_t bo, uint32_t mask, uint32_t sel)
{
    if (NW == 1) {
        r[0] = xor_and(r[0], mask << bo, sel);
        return;
    }
    if (bo < 32) {
        r[0] = xor_and(r[0], mask << bo, sel);
        if (bo > 28) r[NW > 1 ? 1 : 0] = xor_and(r[NW > 1 ? 1 : 0], mask >> (32 - bo), sel);
    } else {
        r[NW > 1 ? 1 : 0] = xor_and(r[NW > 1 ? 1 : 0], mask << (bo - 32), sel);
    }
}

template <int NW>
__device__ void rows_core(const PlanDev *pl, const ChainJob &J, int t_begin, int t_end, uint32_t seed_lo,
                          uint32_t seed_hi, uint8_t *smem)
{
    const int lane = threadIdx.x;
    const int d = (int)uni(pl->d), nq = (int)uni(pl->nq), nblk = (int)uni(pl->nblk);
    const int nranks = (int)uni(pl->nranks), ntypes = (int)uni(pl->ntypes);
    const uint32_t kneg = uni(pl->kneg);
    const int rows = d + 2;
    const int Mpad = 4 * nblk;
    int32_t W[4];
    W[0] = 0; W[1] = (int32_t)uni(pl->W[1]); W[2] = (int32_t)uni(pl->W[2]); W[3] = (int32_t)uni(pl->W[3]);
    const RowsLds lo = rows_layout(ntypes, nranks);
    const uint8_t *lut_s = smem + lo.lut;
    int2 *et_s = reinterpret_cast<int2 *>(__builtin_assume_aligned(smem + lo.et, 8));
    uint32_t *rw = reinterpret_cast<uint32_t *>(smem + lo.rows) + lane;   // this lane's column
    const uint32_t uid = J.uid, cc = J.cc;
    const bool use_x = !J.resume && (J.lp == 1 || J.lp == 2), use_z = !J.resume && (J.lp == 2 || J.lp == 3);

    // pack the state into rows; E of the state on the way
    int32_t E = 0;
    for (int Y = 0; Y < rows; ++Y) {
        const int y = Y - 1;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            uint32_t word = 0;
            if (J.active && y >= 0 && y < d) {
                for (int j = 0; j < 16; ++j) {
                    const int x = 16 * w + j - 1;
                    if (x >= 0 && x < d) {
                        const int q = y * d + x;
                        uint32_t v = J.src[q] & 3u;
                        if (use_x) v ^= pl->lx[q];
                        if (use_z) v ^= pl->lz[q];
                        word |= v << (2 * j);
                        E += weight_of(W, v);
                    }
                }
            }
            rw[(Y * NW + w) * kWave] = word;
        }
    }
    int32_t Emin = E, stop = 0;
    if (J.resume && J.active) {
        E = J.efin[J.ci];
        Emin = J.emin[J.ci];
        stop = J.stop[J.ci];
    }
    wave_lds_fence();

    for (int t = t_begin; t < t_end; ++t) {
        for (int i = lane; i < nranks; i += kWave) et_s[i].y = (int)pl->thr[(size_t)t * nranks + i];
        wave_lds_fence();
        for (int k = 0; k < 4; ++k) {
            // descriptors of class k; the table is padded to a multiple of 4
            const_u32 *tab = (const_u32 *)(uintptr_t)(pl->rowface + k * Mpad);
            int32_t acc_de = 0;
            int curY = -1;
            // rA/rB: the two rows of the current row pair; fA/fB: accumulated
            // flips.  Generators of one class in one row touch disjoint bits,
            // so patterns are read from rA/rB and flips are merged at the end
            // of the row, which keeps the moves of a row independent.
            uint32_t rA[NW], rB[NW], fA[NW], fB[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) rA[w] = rB[w] = fA[w] = fB[w] = 0;
            for (int b = 0; b < nblk; ++b) {
                const uint4 rnd = philox4x32_10(make_uint4(uid, cc, 4u * (uint32_t)t + (uint32_t)k, (uint32_t)b),
                                                seed_lo, seed_hi);
                const uint32_t uw[4] = {rnd.x, rnd.y, rnd.z, rnd.w};
                const uint32_t fdv[4] = {tab[4 * b], tab[4 * b + 1], tab[4 * b + 2], tab[4 * b + 3]};
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    // ranks >= M are null generators (padding bits, dE = 0)
                    const uint32_t fd = fdv[w];
                    const int Y = (int)(fd & 0xFFu);
                    const uint32_t bo = (fd >> 8) & 0xFFu;
                    const uint32_t shp = fd >> 16;
                    if (Y != curY) {
                        if (curY >= 0) {
#pragma unroll
                            for (int v = 0; v < NW; ++v) {
                                rw[(curY * NW + v) * kWave] = rA[v] ^ fA[v];
                                rw[((curY + 1) * NW + v) * kWave] = rB[v] ^ fB[v];
                            }
                        }
#pragma unroll
                        for (int v = 0; v < NW; ++v) {
                            rA[v] = rw[(Y * NW + v) * kWave];
                            rB[v] = rw[((Y + 1) * NW + v) * kWave];
                            fA[v] = fB[v] = 0;
                        }
                        curY = Y;
                    }
                    const uint32_t pat = row_nibble<NW>(rA, bo) | (row_nibble<NW>(rB, bo) << 4);
                    const uint32_t rank = lut_s[(shp << 8) | pat];
                    const int2 et = et_s[rank];
                    // branch-free acceptance: sel is all ones on accepting lanes
                    const bool accept = (rank < kneg) | (uw[w] < (uint32_t)et.y);
                    const uint32_t sel = accept ? 0xFFFFFFFFu : 0u;
                    row_flip_sel<NW>(fA, bo, 6u, sel);   // X_left (2) | Z_up (1 << 2)
                    row_flip_sel<NW>(fB, bo, 9u, sel);   // Z_down (1) | X_right (2 << 2)
                    acc_de += (int32_t)((uint32_t)et.x & sel);
                }
            }
            if (curY >= 0) {
#pragma unroll
                for (int v = 0; v < NW; ++v) {
                    rw[(curY * NW + v) * kWave] = rA[v] ^ fA[v];
                    rw[((curY + 1) * NW + v) * kWave] = rB[v] ^ fB[v];
                }
            }
            wave_lds_fence();
            E += acc_de;
            if (E < Emin) { Emin = E; stop = 4 * t + k + 1; }
        }
    }
    if (J.active) {
        J.emin[J.ci] = Emin;
        J.stop[J.ci] = stop;
        J.efin[J.ci] = E;
        if (J.states) {
            uint8_t *dst = J.states + (size_t)J.ci * nq;
            for (int q = 0; q < nq; ++q) {
                const int y = q / d, x = q - y * d;
                const uint32_t word = rw[((y + 1) * NW + (x + 1) / 16) * kWave];
                dst[q] = (uint8_t)((word >> (2 * ((x + 1) % 16))) & 3u);
            }
        }
    }
    wave_lds_fence();
}

// ---------------------------------------------------------------------------
// Packed-row core specialised to distance D (rotated lattice, D <= 13).
// Same chains as rows_core, bit for bit; what changes is where things live.
// Every row of the chain's padded grid stays in a register for the whole run,
// and the generator schedule (row, nibble offset, shape of every rank of every
// class) is a compile-time table, so the sweep is straight-line code: no
// descriptor loads, no row loads or stores, no per-move scalar work, and the
// null generators that pad a class to whole Philox blocks cost nothing.  The
// move-energy lookup maps (shape, pattern) to the byte offset of a 16-byte
// (dE, threshold, always-accept mask) entry in static LDS; the four generators
// of a Philox block are disjoint, so their patterns are read before any flips.
// ---------------------------------------------------------------------------
__device__ void load_static_tables(const PlanDev *pl, uint16_t *lut_s, uint4 *et_s)
{
    const int lane = threadIdx.x;
    for (int i = lane; i < 256 * 6; i += kWave) lut_s[i] = (uint16_t)(16u * pl->lut[i]);
    for (int i = lane; i < pl->nranks; i += kWave) {
        const int32_t de = pl->dE[i];
        et_s[i] = make_uint4((uint32_t)de, 0u, de <= 0 ? 0xFFFFFFFFu : 0u, 0u);
    }
    wave_lds_fence();
}

// Philox4x32-10 of the counter (uid, cc, c2, b) with uid, c2, b and the key
// uniform across the wavefront and cc the lane's chain.  Tracing which words
// depend on the lane: the two products of round 0 are uniform; round 1
// multiplies one lane word and one uniform word; round 2 likewise; from round
// 3 on every word depends on the lane.  The lane products of rounds 1-2 do
// not involve b, so PhiloxHead computes them once per (sweep, class) and
// philox_block adds the b-dependent uniform products on the scalar unit.
constexpr uint32_t kPhM0 = 0xD2511F53u, kPhM1 = 0xCD9E8D57u, kPhW0 = 0x9E3779B9u, kPhW1 = 0xBB67AE85u;

struct PhiloxHead {
    uint32_t hi0, y1;   // uniform: high word of M0*uid (round 0), low word of M1*c2
    uint32_t w2, z2x;   // lane: round-1 outputs w and (z without the b-dependent part)
    uint32_t a3, y3;    // lane: high and low words of M1*z2 (round 2)
};

__device__ __forceinline__ PhiloxHead philox_head(uint32_t uid, uint32_t cc, uint32_t c2, uint32_t k0, uint32_t k1)
{
    PhiloxHead h;
    const uint64_t p0 = (uint64_t)uid * kPhM0;            // uniform
    const uint64_t p1 = (uint64_t)c2 * kPhM1;             // uniform
    h.hi0 = (uint32_t)(p0 >> 32);
    h.y1 = (uint32_t)p1;
    const uint32_t w1 = (uint32_t)p0;
    const uint32_t x1 = (uint32_t)(p1 >> 32) ^ k0 ^ cc;   // lane
    const uint64_t q = (uint64_t)x1 * kPhM0;              // round 1, lane
    h.z2x = (uint32_t)(q >> 32) ^ w1 ^ (k1 + kPhW1);
    h.w2 = (uint32_t)q;
    const uint64_t r = (uint64_t)h.z2x * kPhM1;           // round 2, lane
    h.a3 = (uint32_t)(r >> 32);
    h.y3 = (uint32_t)r;
    return h;
}

__device__ __forceinline__ uint4 philox_block(const PhiloxHead &h, uint32_t b, uint32_t k0, uint32_t k1)
{
    uint32_t z1 = h.hi0 ^ b ^ k1;                         // round 0 output z (uniform)
    // computed per block on the scalar unit rather than hoisted out of the
    // sweep loop into vector registers
    asm volatile("" : "+s"(z1));
    const uint64_t p1 = (uint64_t)z1 * kPhM1;             // round 1, uniform
    const uint32_t x2 = (uint32_t)(p1 >> 32) ^ h.y1 ^ (k0 + kPhW0);
    const uint32_t y2 = (uint32_t)p1;
    const uint64_t p0 = (uint64_t)x2 * kPhM0;             // round 2, uniform
    uint4 c = make_uint4(h.a3 ^ (y2 ^ (k0 + 2u * kPhW0)), h.y3,
                         h.w2 ^ ((uint32_t)(p0 >> 32) ^ (k1 + 2u * kPhW1)), (uint32_t)p0);
    k0 += 3u * kPhW0;
    k1 += 3u * kPhW1;
#pragma unroll
    for (int i = 3; i < 10; ++i) {
        const uint64_t q0 = (uint64_t)c.x * kPhM0;
        const uint64_t q1 = (uint64_t)c.z * kPhM1;
        c = make_uint4(xor3_key((uint32_t)(q1 >> 32), c.y, k0), (uint32_t)q1,
                       xor3_key((uint32_t)(q0 >> 32), c.w, k1), (uint32_t)q0);
        k0 += kPhW0;
        k1 += kPhW1;
    }
    return c;
}

// All ones where u < thr (unsigned), from the borrow of u - thr: bit 31 of
// (~u & thr) | (~(u ^ thr) & (u - thr)), one v_bitop3 (truth table 0x8E).
__device__ __forceinline__ uint32_t lt_mask(uint32_t u, uint32_t thr)
{
    return (uint32_t)((int32_t)__builtin_amdgcn_bitop3_b32(u, thr, u - thr, 0x8E) >> 31);
}

// Pattern of the generator at nibble offset BO of rows (ra, rb), times two:
// bits 1-4 from ra, bits 5-8 from rb.
template <int BO>
__device__ __forceinline__ uint32_t pattern_x2(uint32_t ra, uint32_t rb)
{
    const uint32_t a = BO >= 1 ? ra >> (BO - 1) : ra << 1;
    const uint32_t b = BO >= 5 ? rb >> (BO - 5) : rb << (5 - BO);
    return (b & 0x1E0u) | (a & 0x1Eu);
}

template <int D, int K, int B, int W>
__device__ __forceinline__ void static_move(uint32_t (&r)[D + 2], uint32_t u, const uint16_t *lut_s, const uint4 *et_s,
                                            int32_t &acc)
{
    constexpr RotSchedule<D> S{};
    constexpr RotGen g = S.g[K][4 * B + W];
    if constexpr (g.shp != 5) {
        const uint32_t pat2 = pattern_x2<g.bo>(r[g.Y], r[g.Y + 1]);
        const uint32_t off = *reinterpret_cast<const uint16_t *>(reinterpret_cast<const uint8_t *>(lut_s) +
                                                                 512u * g.shp + pat2);
        const uint4 e = *reinterpret_cast<const uint4 *>(reinterpret_cast<const uint8_t *>(et_s) + off);
        // all ones on accepting lanes: u < threshold, or dE <= 0
        const uint32_t sel = lt_mask(u, e.y) | e.z;
        r[g.Y] = xor_and(r[g.Y], 6u << g.bo, sel);           // X_left | Z_up
        r[g.Y + 1] = xor_and(r[g.Y + 1], 9u << g.bo, sel);   // Z_down | X_right
        acc += (int32_t)(e.x & sel);
    }
}

template <int D, int K, int B>
__device__ __forceinline__ void static_block(uint32_t (&r)[D + 2], const PhiloxHead &h, uint32_t k0, uint32_t k1,
                                             const uint16_t *lut_s, const uint4 *et_s, int32_t &acc)
{
    const uint4 u = philox_block(h, (uint32_t)B, k0, k1);
    static_move<D, K, B, 0>(r, u.x, lut_s, et_s, acc);
    static_move<D, K, B, 1>(r, u.y, lut_s, et_s, acc);
    static_move<D, K, B, 2>(r, u.z, lut_s, et_s, acc);
    static_move<D, K, B, 3>(r, u.w, lut_s, et_s, acc);
}

template <int D, int K, int... Bs>
__device__ __forceinline__ void static_class(uint32_t (&r)[D + 2], const PhiloxHead &h, uint32_t k0, uint32_t k1,
                                             const uint16_t *lut_s, const uint4 *et_s, int32_t &acc,
                                             std::integer_sequence<int, Bs...>)
{
    (static_block<D, K, Bs>(r, h, k0, k1, lut_s, et_s, acc), ...);
}

template <int D>
__device__ void rows_static_core(const PlanDev *pl, const ChainJob &J, int t_begin, int t_end, uint32_t seed_lo,
                                 uint32_t seed_hi, const uint16_t *lut_s, uint4 *et_s, int cp_interval)
{
    constexpr int NR = D + 2;
    constexpr int NB = RotSchedule<D>::MP / 4;
    using Blocks = std::make_integer_sequence<int, NB>;
    const int lane = threadIdx.x;
    const int nranks = (int)uni(pl->nranks);
    int32_t W[4];
    W[0] = 0; W[1] = (int32_t)uni(pl->W[1]); W[2] = (int32_t)uni(pl->W[2]); W[3] = (int32_t)uni(pl->W[3]);
    // a task's 64 chains belong to one syndrome
    const uint32_t uid = uni(J.uid), cc = J.cc;
    const uint32_t k0 = uni(seed_lo), k1 = uni(seed_hi);
    const bool use_x = !J.resume && (J.lp == 1 || J.lp == 2), use_z = !J.resume && (J.lp == 2 || J.lp == 3);
    // lane 0 is always active and a task's chains are consecutive: chain of lane l = ci0 + l
    const int64_t ci0 = (int64_t)(((uint64_t)uni((uint32_t)((uint64_t)J.ci >> 32)) << 32) | uni((uint32_t)J.ci));
    const int cp_every = J.cp_out ? cp_interval : 0;

    uint32_t r[NR];
    int32_t E = 0;
#pragma unroll
    for (int Y = 0; Y < NR; ++Y) {
        uint32_t word = 0;
        if (Y >= 1 && Y <= D && J.active) {
            // not unrolled: a fully unrolled row would keep every byte load in flight
#pragma unroll 1
            for (int x = 0; x < D; ++x) {
                const int q = (Y - 1) * D + x;
                uint32_t v = J.src[q] & 3u;
                if (use_x) v ^= pl->lx[q];
                if (use_z) v ^= pl->lz[q];
                word |= v << (2 * (x + 1));
                E += weight_of(W, v);
            }
        }
        r[Y] = word;
    }
    int32_t Emin = E, stop = 0;
    if (J.resume && J.active) {
        E = J.efin[J.ci];
        Emin = J.emin[J.ci];
        stop = J.stop[J.ci];
    }

    for (int t = t_begin; t < t_end;) {
        // sweeps up to the next checkpoint, then the checkpoint (the state at
        // the start of sweep t, every cp_every sweeps)
        int t_stop = t_end;
        if (cp_every) t_stop = min(t_end, (t / cp_every + 1) * cp_every);
        for (; t < t_stop; ++t) {
            wave_lds_fence();
            for (int i = lane; i < nranks; i += kWave) et_s[i].y = pl->thr[(size_t)t * nranks + i];
            wave_lds_fence();
            const uint32_t c2 = 4u * (uint32_t)t;
            int32_t acc = 0;
            static_class<D, 0>(r, philox_head(uid, cc, c2, k0, k1), k0, k1, lut_s, et_s, acc, Blocks{});
            E += acc;
            if (E < Emin) { Emin = E; stop = 4 * t + 1; }
            acc = 0;
            static_class<D, 1>(r, philox_head(uid, cc, c2 + 1u, k0, k1), k0, k1, lut_s, et_s, acc, Blocks{});
            E += acc;
            if (E < Emin) { Emin = E; stop = 4 * t + 2; }
            acc = 0;
            static_class<D, 2>(r, philox_head(uid, cc, c2 + 2u, k0, k1), k0, k1, lut_s, et_s, acc, Blocks{});
            E += acc;
            if (E < Emin) { Emin = E; stop = 4 * t + 3; }
            acc = 0;
            static_class<D, 3>(r, philox_head(uid, cc, c2 + 3u, k0, k1), k0, k1, lut_s, et_s, acc, Blocks{});
            E += acc;
            if (E < Emin) { Emin = E; stop = 4 * t + 4; }
        }
        if (cp_every && t < t_end && J.active) {
            uint32_t *cp = J.cp_out + (int64_t)(t / cp_every - 1) * D * J.cp_stride + ci0 + lane;
#pragma unroll
            for (int Y = 1; Y <= D; ++Y) cp[(Y - 1) * J.cp_stride] = r[Y];
        }
    }
    if (J.active) {
        J.emin[J.ci] = Emin;
        J.stop[J.ci] = stop;
        J.efin[J.ci] = E;
        if (J.states) {
            uint8_t *dst = J.states + (size_t)J.ci * (D * D);
#pragma unroll
            for (int Y = 1; Y <= D; ++Y)
#pragma unroll 1
                for (int x = 0; x < D; ++x) dst[(Y - 1) * D + x] = (uint8_t)((r[Y] >> (2 * (x + 1))) & 3u);
        }
    }
}

__device__ void load_rows_tables(const PlanDev *pl, uint8_t *smem)
{
    const int lane = threadIdx.x;
    const RowsLds lo = rows_layout(pl->ntypes, pl->nranks);
    const uint32_t *lut_g = reinterpret_cast<const uint32_t *>(pl->lut);
    uint32_t *lut_s = reinterpret_cast<uint32_t *>(smem + lo.lut);
    for (int i = lane; i < 64 * pl->ntypes; i += kWave) lut_s[i] = lut_g[i];
    int2 *et_s = reinterpret_cast<int2 *>(smem + lo.et);
    for (int i = lane; i < pl->nranks; i += kWave) et_s[i] = make_int2(pl->dE[i], 0);
    wave_lds_fence();
}

__device__ void load_plan_tables(const PlanDev *pl, uint8_t *smem)
{
    const int lane = threadIdx.x;
    const LdsLayout lo = lds_layout(pl->M, pl->ntypes, pl->nranks);
    uint2 *desc_s = reinterpret_cast<uint2 *>(smem + lo.desc);
    const uint2 *desc_g = reinterpret_cast<const uint2 *>(pl->desc);
    for (int i = lane; i < 4 * pl->M; i += kWave) desc_s[i] = desc_g[i];
    const uint32_t *lut_g = reinterpret_cast<const uint32_t *>(pl->lut);
    uint32_t *lut_s = reinterpret_cast<uint32_t *>(smem + lo.lut);
    for (int i = lane; i < 64 * pl->ntypes; i += kWave) lut_s[i] = lut_g[i];
    int2 *et_s = reinterpret_cast<int2 *>(smem + lo.et);
    for (int i = lane; i < pl->nranks; i += kWave) et_s[i] = make_int2(pl->dE[i], 0);
    wave_lds_fence();
}

// ---------------------------------------------------------------------------
// Batch kernels.  MODE 0: persistent wavefronts pulling tasks from an atomic
// queue over every group of the launch; MODE 2: plain form, one task per
// workgroup.  ROWS selects the packed-row core; otherwise the byte-state core
// with LOGG = log2(lanes per chain), the same for every group of the launch;
// REPLAY (byte-state only) re-runs each syndrome's best chain.
// ---------------------------------------------------------------------------
template <int MODE, bool ROWS, int LOGG, bool REPLAY>
__device__ __forceinline__ void batch_kernel_body(const AnnealArgs &A)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const PlanDev *loaded = nullptr;
    for (int iter = 0;; ++iter) {
        uint32_t task = 0;
        if (MODE == 2) {
            if (iter > 0) break;
            task = blockIdx.x;
        } else {
            if (threadIdx.x == 0) task = atomicAdd(A.counter, 1u);
            task = __builtin_amdgcn_readfirstlane(__shfl(task, 0, kWave));
        }
        if (task >= A.n_tasks) break;
        int gi = 0;
        while (gi + 1 < A.n_groups && (int64_t)task >= A.g[gi + 1].task_begin) ++gi;
        const GroupArgs &G = A.g[gi];
        constexpr int lg = ROWS ? 0 : LOGG;
        const int64_t unit0 = ((int64_t)task - G.task_begin) << (6 - lg);
        if (G.plan != loaded) {
            wave_lds_fence();
            if (ROWS) load_rows_tables(G.plan, smem);
            else load_plan_tables(G.plan, smem);
            loaded = G.plan;
        }
        const int n_sweeps = G.plan->n_sweeps;
        if (ROWS) {
            const ChainJob J = batch_job(G, unit0 + threadIdx.x, false);
            if (G.row_words == 1) rows_core<1>(G.plan, J, 0, n_sweeps, A.seed_lo, A.seed_hi, smem);
            else rows_core<2>(G.plan, J, 0, n_sweeps, A.seed_lo, A.seed_hi, smem);
        } else {
            const ChainJob J = batch_job(G, unit0 + (threadIdx.x >> lg), REPLAY);
            // a replay from a checkpoint runs one chain per wavefront (uniform t0)
            bytes_core<lg, REPLAY>(G.plan, J, REPLAY ? J.t0 : 0, n_sweeps, A.seed_lo, A.seed_hi, smem);
        }
    }
}

// Batch body of the specialised packed-row kernel (MODE as above).  Every
// group of the launch has distance SD and tasks of 64 chains of one syndrome.
template <int MODE, int SD>
__device__ __forceinline__ void static_rows_body(const AnnealArgs &A)
{
    __shared__ uint16_t lut_s[256 * 6];
    __shared__ uint4 et_s[kStaticRanks];
    const PlanDev *loaded = nullptr;
    for (int iter = 0;; ++iter) {
        uint32_t task = 0;
        if (MODE == 2) {
            if (iter > 0) break;
            task = blockIdx.x;
        } else {
            if (threadIdx.x == 0) task = atomicAdd(A.counter, 1u);
            task = __builtin_amdgcn_readfirstlane(__shfl(task, 0, kWave));
        }
        if (task >= A.n_tasks) break;
        int gi = 0;
        while (gi + 1 < A.n_groups && (int64_t)task >= A.g[gi + 1].task_begin) ++gi;
        const GroupArgs &G = A.g[gi];
        const int64_t unit0 = ((int64_t)task - G.task_begin) << 6;
        if (G.plan != loaded) {
            wave_lds_fence();
            load_static_tables(G.plan, lut_s, et_s);
            loaded = G.plan;
        }
        const ChainJob J = batch_job(G, unit0 + threadIdx.x, false);
        rows_static_core<SD>(G.plan, J, 0, G.plan->n_sweeps, A.seed_lo, A.seed_hi, lut_s, et_s, G.cp_every);
    }
}

// Occupancy target of the specialised kernels: eight wavefronts per SIMD (at
// most 64 VGPRs) hides the LDS and multiply latencies best, even at the cost
// of a few spilled registers at d = 11 (measured); d = 13 keeps six.
constexpr int static_waves(int d) { return d <= 11 ? 8 : 6; }

template <int D>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(static_waves(D), static_waves(D))))
void k_anneal_rows_d(AnnealArgs A) { static_rows_body<0, D>(A); }
template <int D>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(static_waves(D), static_waves(D))))
void k_anneal_rows_d_plain(AnnealArgs A) { static_rows_body<2, D>(A); }

template <int LOGG>
__global__ __launch_bounds__(kWave) void k_anneal(AnnealArgs A) { batch_kernel_body<0, false, LOGG, false>(A); }
template <int LOGG>
__global__ __launch_bounds__(kWave) void k_replay(AnnealArgs A) { batch_kernel_body<0, false, LOGG, true>(A); }
template <int LOGG>
__global__ __launch_bounds__(kWave) void k_anneal_plain(AnnealArgs A) { batch_kernel_body<2, false, LOGG, false>(A); }
__global__ __launch_bounds__(kWave) void k_anneal_rows(AnnealArgs A) { batch_kernel_body<0, true, 0, false>(A); }
__global__ __launch_bounds__(kWave) void k_anneal_rows_plain(AnnealArgs A) { batch_kernel_body<2, true, 0, false>(A); }

typedef void (*AnnealKernel)(AnnealArgs);
static AnnealKernel static_rows_kernel(int d, bool plain)
{
    switch (d) {
    case 3: return plain ? k_anneal_rows_d_plain<3> : k_anneal_rows_d<3>;
    case 5: return plain ? k_anneal_rows_d_plain<5> : k_anneal_rows_d<5>;
    case 7: return plain ? k_anneal_rows_d_plain<7> : k_anneal_rows_d<7>;
    case 9: return plain ? k_anneal_rows_d_plain<9> : k_anneal_rows_d<9>;
    case 11: return plain ? k_anneal_rows_d_plain<11> : k_anneal_rows_d<11>;
    case 13: return plain ? k_anneal_rows_d_plain<13> : k_anneal_rows_d<13>;
    default: return nullptr;
    }
}

static AnnealKernel bytes_kernel(int mode, int lg)
{
    // mode 0: persistent, 1: replay, 2: plain
    static const AnnealKernel tab[3][7] = {
        {k_anneal<0>, k_anneal<1>, k_anneal<2>, k_anneal<3>, k_anneal<4>, k_anneal<5>, k_anneal<6>},
        {k_replay<0>, k_replay<1>, k_replay<2>, k_replay<3>, k_replay<4>, k_replay<5>, k_replay<6>},
        {k_anneal_plain<0>, k_anneal_plain<1>, k_anneal_plain<2>, k_anneal_plain<3>, k_anneal_plain<4>,
         k_anneal_plain<5>, k_anneal_plain<6>}};
    return tab[mode][lg];
}

// ---------------------------------------------------------------------------
// Serving kernels: one workgroup per task of the slice.  A task covers
// consecutive chains of one resident request, all at the same sweep range.
// ---------------------------------------------------------------------------

__device__ __forceinline__ ChainJob serve_job(const ServeTask &T, int slot, bool replay)
{
    ChainJob j;
    const int nc = 4 * T.n_rep;
    const int nq = T.plan->nq;
    j.active = slot < T.nchains;
    int c = T.chain0 + (j.active ? slot : 0);
    if (replay) c = *T.best;
    j.cc = (uint32_t)c;
    j.lp = c & 3;
    j.uid = T.uid;
    j.resume = !replay && T.t_begin > 0;
    j.src = j.resume ? T.states + (size_t)c * nq : T.refs + (size_t)(c >> 2) * nq;
    j.ci = c;
    j.efin = T.e3;
    j.emin = T.e3 + nc;
    j.stop = T.e3 + 2 * nc;
    j.states = replay ? nullptr : T.states;
    j.target = replay ? T.e3[2 * nc + c] : -1;
    j.snap = replay ? T.snap : nullptr;
    j.cp_out = nullptr;
    j.cp_in = nullptr;
    j.cp_stride = 0;
    j.t0 = 0;
    return j;
}

template <bool ROWS, bool REPLAY>
__device__ __forceinline__ void serve_kernel_body(const ServeTask *tasks, uint32_t seed_lo, uint32_t seed_hi)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const ServeTask &T = tasks[blockIdx.x];
    const PlanDev *pl = T.plan;
    if (ROWS) {
        load_rows_tables(pl, smem);
        const ChainJob J = serve_job(T, threadIdx.x, false);
        if (T.row_words == 1) rows_core<1>(pl, J, T.t_begin, T.t_end, seed_lo, seed_hi, smem);
        else rows_core<2>(pl, J, T.t_begin, T.t_end, seed_lo, seed_hi, smem);
    } else {
        load_plan_tables(pl, smem);
        const int lg = T.log_lanes;
        const ChainJob J = serve_job(T, threadIdx.x >> lg, REPLAY);
        const int tb = REPLAY ? 0 : T.t_begin;
        const int te = REPLAY ? pl->n_sweeps : T.t_end;
        switch (lg) {
        case 0: bytes_core<0, REPLAY>(pl, J, tb, te, seed_lo, seed_hi, smem); break;
        case 1: bytes_core<1, REPLAY>(pl, J, tb, te, seed_lo, seed_hi, smem); break;
        case 2: bytes_core<2, REPLAY>(pl, J, tb, te, seed_lo, seed_hi, smem); break;
        case 3: bytes_core<3, REPLAY>(pl, J, tb, te, seed_lo, seed_hi, smem); break;
        case 4: bytes_core<4, REPLAY>(pl, J, tb, te, seed_lo, seed_hi, smem); break;
        case 5: bytes_core<5, REPLAY>(pl, J, tb, te, seed_lo, seed_hi, smem); break;
        default: bytes_core<6, REPLAY>(pl, J, tb, te, seed_lo, seed_hi, smem); break;
        }
    }
}

__global__ __launch_bounds__(kWave) void k_serve_rows(const ServeTask *tasks, uint32_t slo, uint32_t shi)
{
    serve_kernel_body<true, false>(tasks, slo, shi);
}
__global__ __launch_bounds__(kWave) void k_serve_bytes(const ServeTask *tasks, uint32_t slo, uint32_t shi)
{
    serve_kernel_body<false, false>(tasks, slo, shi);
}
__global__ __launch_bounds__(kWave) void k_serve_replay(const ServeTask *tasks, uint32_t slo, uint32_t shi)
{
    serve_kernel_body<false, true>(tasks, slo, shi);
}

__global__ void k_zero_u32(uint32_t *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Reduction (Alg. 7, Eq. (21)) -- one wavefront per syndrome.  Chain c of
// replica r = c/4 runs in coset Q_r * P' (P' = c mod 4); E_P is the minimum
// E_min over the chains of coset P; P* = argmin with ties to the lowest index;
// the best chain is the lowest chain of coset P* attaining E_P*.
// ---------------------------------------------------------------------------
struct ReduceArgs {
    const PlanDev *plan;
    const uint8_t *qcls;
    const uint8_t *refs;
    const int32_t *emin;
    int32_t *e_best;
    uint8_t *cls;
    int32_t *best_chain;
    int32_t *e_cls;
    uint8_t *paper_recovery;
    int64_t n_syn;
    int n_rep;
};

__global__ __launch_bounds__(kWave) void k_reduce(ReduceArgs A)
{
    const int lane = threadIdx.x;
    const int64_t s = blockIdx.x;
    const int nc = 4 * A.n_rep;
    uint64_t best[4] = {~0ull, ~0ull, ~0ull, ~0ull};
    for (int c = lane; c < nc; c += kWave) {
        const int cls = cls_mul(A.qcls[s * A.n_rep + (c >> 2)], c & 3);
        const uint64_t key = ((uint64_t)(uint32_t)A.emin[s * nc + c] << 32) | (uint32_t)c;
#pragma unroll
        for (int P = 0; P < 4; ++P)
            if (cls == P) best[P] = min(best[P], key);
    }
#pragma unroll
    for (int P = 0; P < 4; ++P)
#pragma unroll
        for (int sh = 1; sh < kWave; sh <<= 1) {
            const uint64_t o = __shfl_xor(best[P], sh, kWave);
            best[P] = min(best[P], o);
        }
    int ps = 0;
#pragma unroll
    for (int P = 1; P < 4; ++P)
        if ((best[P] >> 32) < (best[ps] >> 32)) ps = P;
    if (lane == 0) {
        A.e_best[s] = (int32_t)(best[ps] >> 32);
        A.cls[s] = (uint8_t)ps;
        A.best_chain[s] = (int32_t)(best[ps] & 0xFFFFFFFFu);
        if (A.e_cls)
            for (int P = 0; P < 4; ++P) A.e_cls[s * 4 + P] = best[P] == ~0ull ? INT32_MAX : (int32_t)(best[P] >> 32);
    }
    if (A.paper_recovery) {
        const PlanDev *pl = A.plan;
        const int nq = pl->nq;
        const bool ux = (ps == 1 || ps == 2), uz = (ps == 2 || ps == 3);
        const uint8_t *r0 = A.refs + (size_t)s * A.n_rep * nq;
        for (int q = lane; q < nq; q += kWave)
            A.paper_recovery[(size_t)s * nq + q] = r0[q] ^ (ux ? pl->lx[q] : 0) ^ (uz ? pl->lz[q] : 0);
    }
}

// Serving: per-coset reduction of a finished request (one wavefront each).
// The class of replica r relative to replica 0 comes from the raw symplectic
// bits the greedy kernel stored (bit 0: with L_Z, bit 1: with L_X).
__global__ __launch_bounds__(kWave) void k_serve_reduce(const ServeFinish *fin)
{
    const ServeFinish &F = fin[blockIdx.x];
    const int lane = threadIdx.x;
    const int nc = 4 * F.n_rep;
    const int raw0 = F.qraw[0] & 3;
    uint64_t best[4] = {~0ull, ~0ull, ~0ull, ~0ull};
    for (int c = lane; c < nc; c += kWave) {
        const int v = (F.qraw[c >> 2] & 3) ^ raw0;
        const int cls = cls_mul(cls_from_bits(v & 1, v >> 1), c & 3);
        const uint64_t key = ((uint64_t)(uint32_t)F.e3[nc + c] << 32) | (uint32_t)c;
#pragma unroll
        for (int P = 0; P < 4; ++P)
            if (cls == P) best[P] = min(best[P], key);
    }
#pragma unroll
    for (int P = 0; P < 4; ++P)
#pragma unroll
        for (int sh = 1; sh < kWave; sh <<= 1) best[P] = min(best[P], (uint64_t)__shfl_xor(best[P], sh, kWave));
    int ps = 0;
#pragma unroll
    for (int P = 1; P < 4; ++P)
        if ((best[P] >> 32) < (best[ps] >> 32)) ps = P;
    if (lane == 0) {
        F.result[0] = (int32_t)(best[ps] >> 32);
        F.result[1] = ps;
        F.result[2] = (int32_t)(best[ps] & 0xFFFFFFFFu);
        for (int P = 0; P < 4; ++P) F.result[4 + P] = best[P] == ~0ull ? INT32_MAX : (int32_t)(best[P] >> 32);
    }
}

// ---------------------------------------------------------------------------
// Host-side launch logic.
// ---------------------------------------------------------------------------
static int check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return XZZX_OK;
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return XZZX_EDEVICE;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static int greedy_lds(const Plan &P, int *max_nodes)
{
    const int mn = std::max(P.hdev.ncol[0], P.hdev.ncol[1]);
    *max_nodes = mn;
    return 4 * ((P.lat.nq + 3) / 4) + 3 * 4 * (mn + 1) + (mn + 1) + 16;
}

static int launch_greedy(const Plan &P, const uint8_t *d_syn, const uint32_t *d_uid, int64_t n_syn,
                         int n_rep, uint64_t seed, int mode, uint8_t *d_refs, uint8_t *d_qraw,
                         hipStream_t stream)
{
    if (n_syn == 0) return XZZX_OK;
    GreedyArgs A{};
    A.plan = P.ddev;
    A.syn = d_syn;
    A.uid = d_uid;
    A.refs = d_refs;
    A.qraw = d_qraw;
    A.n_syn = n_syn;
    A.n_rep = n_rep;
    A.mode = mode;
    A.syn_stride = P.lat.nstab;
    A.seed_lo = (uint32_t)seed;
    A.seed_hi = (uint32_t)(seed >> 32);
    const int lds = greedy_lds(P, &A.max_nodes);
    const int64_t blocks = n_syn * n_rep;
    if (blocks > 0x7FFFFFFF) { set_error("too many (syndrome, replica) pairs"); return XZZX_ERANGE; }
    hipLaunchKernelGGL(k_greedy, dim3((unsigned)blocks), dim3(kWave), lds, stream, A);
    return check_hip(hipGetLastError(), "k_greedy launch");
}

static int launch_qcls(const uint8_t *d_qraw, int64_t n_syn, int n_rep, uint8_t *d_qcls, hipStream_t stream)
{
    if (n_syn == 0) return XZZX_OK;
    hipLaunchKernelGGL(k_qcls, dim3((unsigned)((n_syn + 255) / 256)), dim3(256), 0, stream, d_qraw, n_syn, n_rep, d_qcls);
    return check_hip(hipGetLastError(), "k_qcls launch");
}

// Per-group workspace layout.
struct GroupWs {
    uint8_t *refs, *qraw, *qcls;
    int32_t *emin, *stop, *efin, *best_chain;
    uint32_t *cp_rows;     // checkpoints of groups on the specialised packed-row kernel
};

// A group runs on the packed-row kernel specialised to its distance when the
// plan allows it and every 64-chain task lies inside one syndrome.
static bool uses_static(const xzzx_group &g, int64_t unit_offset)
{
    const Plan &P = g.plan->P;
    return P.use_rows && P.static_d && (4 * g.n_rep) % kWave == 0 && unit_offset % kWave == 0;
}

// Checkpoints a specialised group keeps: the states at the start of sweeps
// kCheckpointEvery, 2 kCheckpointEvery, ... before the last sweep.
static int checkpoints_of(const xzzx_group &g)
{
    if (!uses_static(g, 0) || g.plan->P.n_sweeps <= 0) return 0;
    return (g.plan->P.n_sweeps - 1) / kCheckpointEvery;
}

static size_t group_ws_bytes(const xzzx_group &g, bool decode)
{
    const Plan &P = g.plan->P;
    const size_t nq = P.lat.nq, ns = (size_t)g.n_syn, R = (size_t)g.n_rep, nc = 4 * R * ns;
    size_t b = 0;
    if (decode && !g.d_refs) b += align256(ns * R * nq);
    b += align256(ns * R);                                  // qraw
    if (decode && !g.d_qcls) b += align256(ns * R);
    if (!g.d_chain_emin) b += align256(nc * 4);
    if (!g.d_chain_stop) b += align256(nc * 4);
    if (!g.d_chain_e) b += align256(nc * 4);
    if (!g.d_best_chain) b += align256(ns * 4);
    b += align256((size_t)checkpoints_of(g) * P.lat.d * nc * 4);
    return b;
}

static GroupWs carve_group(const xzzx_group &g, bool decode, uint8_t *&p)
{
    const Plan &P = g.plan->P;
    const size_t nq = P.lat.nq, ns = (size_t)g.n_syn, R = (size_t)g.n_rep, nc = 4 * R * ns;
    GroupWs w{};
    auto take = [&](size_t bytes) { uint8_t *r = p; p += align256(bytes); return r; };
    w.refs = g.d_refs ? g.d_refs : (decode ? take(ns * R * nq) : nullptr);
    w.qraw = take(ns * R);
    w.qcls = g.d_qcls ? g.d_qcls : (decode ? take(ns * R) : nullptr);
    w.emin = g.d_chain_emin ? g.d_chain_emin : reinterpret_cast<int32_t *>(take(nc * 4));
    w.stop = g.d_chain_stop ? g.d_chain_stop : reinterpret_cast<int32_t *>(take(nc * 4));
    w.efin = g.d_chain_e ? g.d_chain_e : reinterpret_cast<int32_t *>(take(nc * 4));
    w.best_chain = g.d_best_chain ? g.d_best_chain : reinterpret_cast<int32_t *>(take(ns * 4));
    const int ncp = checkpoints_of(g);
    w.cp_rows = ncp ? reinterpret_cast<uint32_t *>(take((size_t)ncp * P.lat.d * nc * 4)) : nullptr;
    return w;
}

static int validate_groups(const xzzx_group *groups, int n_groups, bool decode)
{
    if (!groups || n_groups < 1 || n_groups > kMaxGroups) {
        set_error("need 1..16 groups");
        return XZZX_EINVAL;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { set_error("hipGetDevice failed"); return XZZX_EDEVICE; }
    for (int i = 0; i < n_groups; ++i) {
        const xzzx_group &g = groups[i];
        if (!g.plan || g.n_syn < 0 || g.n_rep < 1 || g.n_rep > (1 << 20)) { set_error("bad group (plan, n_syn or n_rep)"); return XZZX_EINVAL; }
        if (g.plan->P.device != dev) { set_error("plan was created on another device"); return XZZX_EINVAL; }
        if (g.n_syn == 0) continue;
        if (!g.d_uid || !g.d_e_best || !g.d_cls || !g.d_recovery) { set_error("missing required group buffer"); return XZZX_EINVAL; }
        if (decode && !g.d_syn) { set_error("decode needs d_syn"); return XZZX_EINVAL; }
        if (!decode && (!g.d_refs || !g.d_qcls)) { set_error("anneal needs d_refs and d_qcls"); return XZZX_EINVAL; }
        if ((int64_t)g.n_syn * 4 * g.n_rep >= ((int64_t)1 << 31)) { set_error("too many chains in one group"); return XZZX_ERANGE; }
    }
    return XZZX_OK;
}

static int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    return cus;
}

static int anneal_grid(const void *kernel, size_t lds_bytes, uint32_t n_tasks, unsigned *grid)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWave, lds_bytes) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    const uint64_t full = (uint64_t)device_cus() * (uint64_t)per_cu;
    *grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(full, n_tasks));
    return XZZX_OK;
}

static int log2_int(int v)
{
    int lg = 0;
    while ((1 << lg) < v) ++lg;
    return lg;
}

enum class AnnealMode { Persistent, Replay, Plain };

// Launch one annealing kernel over `units` of the selected groups (chains, or
// syndromes in replay mode).  rows: packed-row kernel (one chain per lane);
// otherwise the byte-state kernel with the plan's lanes per chain.  The replay
// re-runs one chain per syndrome with the byte-state kernel, spreading a chain
// over more lanes when that is needed to give every CU several wavefronts.
static int launch_set(const xzzx_group *groups, const GroupWs *ws, const std::vector<int> &sel, bool rows, int lanes,
                      AnnealMode mode, uint64_t seed, int64_t unit_offset, int64_t units_override,
                      uint32_t *d_counter, hipStream_t stream, int static_d = 0)
{
    const bool replay = mode == AnnealMode::Replay;
    AnnealArgs A{};
    A.seed_lo = (uint32_t)seed;
    A.seed_hi = (uint32_t)(seed >> 32);
    A.counter = d_counter;
    auto units_of = [&](int i) -> int64_t {
        return units_override >= 0 ? units_override : (replay ? groups[i].n_syn : groups[i].n_syn * 4 * groups[i].n_rep);
    };
    // order groups by work per task (largest first) so the queue is LPT-like
    std::vector<int> order = sel;
    auto cost = [&](int i) {
        const Plan &P = groups[i].plan->P;
        return (double)P.n_sweeps * P.lat.nstab;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    uint64_t tasks = 0;
    size_t lds = 0;
    int ng = 0;
    const int lg = log2_int(lanes);
    for (int i : order) {
        const xzzx_group &g = groups[i];
        const Plan &P = g.plan->P;
        GroupArgs &G = A.g[ng++];
        G.plan = P.ddev;
        G.uid = g.d_uid;
        G.refs = ws[i].refs;
        G.emin = ws[i].emin;
        G.stop = ws[i].stop;
        G.efin = ws[i].efin;
        G.final = replay ? nullptr : g.d_chain_final;
        G.best_chain = ws[i].best_chain;
        G.recovery = g.d_recovery;
        G.n_rep = g.n_rep;
        G.log_lanes = lg;
        G.row_words = rows ? P.row_words : 0;
        // checkpoints: written by the specialised kernel, read by the replay
        const bool cp = checkpoints_of(g) > 0 && (static_d || replay);
        G.cp_rows = cp ? ws[i].cp_rows : nullptr;
        G.cp_every = cp ? kCheckpointEvery : 0;
        G.n_chains = g.n_syn * 4 * g.n_rep;
        G.unit_offset = unit_offset;
        const int64_t units = units_of(i);
        G.n_units = units;
        G.task_begin = (int64_t)tasks;
        const int C = kWave / lanes;
        tasks += (uint64_t)((units + C - 1) / C);
        lds = std::max(lds, static_d ? (size_t)0 : rows ? P.lds_bytes_rows() : P.lds_bytes_anneal(lanes));
    }
    if (ng == 0 || tasks == 0) return XZZX_OK;
    if (tasks >= 0xFFFFFFF0ull) { set_error("too many anneal tasks in one launch"); return XZZX_ERANGE; }
    A.n_groups = ng;
    A.n_tasks = (uint32_t)tasks;
    if (lds > 65536) { set_error("LDS demand above 64 KiB"); return XZZX_ERANGE; }
    if (mode == AnnealMode::Plain) {
        if (static_d)
            hipLaunchKernelGGL(static_rows_kernel(static_d, true), dim3((unsigned)tasks), dim3(kWave), 0, stream, A);
        else if (rows)
            hipLaunchKernelGGL(k_anneal_rows_plain, dim3((unsigned)tasks), dim3(kWave), lds, stream, A);
        else
            hipLaunchKernelGGL(bytes_kernel(2, lg), dim3((unsigned)tasks), dim3(kWave), lds, stream, A);
        return check_hip(hipGetLastError(), "plain anneal launch");
    }
    const AnnealKernel kern =
        static_d ? static_rows_kernel(static_d, false) : rows ? k_anneal_rows : bytes_kernel(replay ? 1 : 0, lg);
    unsigned grid = 0;
    int rc = anneal_grid((const void *)kern, lds, A.n_tasks, &grid);
    if (rc) return rc;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, stream, d_counter, 1);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWave), lds, stream, A);
    return check_hip(hipGetLastError(), "anneal launch");
}

// Annealing of every non-empty group.  Packed-row groups share one persistent
// launch; byte-state groups are launched per lanes-per-chain value.  The
// replay re-runs one chain per syndrome with the byte-state kernel, spreading
// a chain over more lanes when that is needed to give every CU several
// wavefronts.  Each launch has its own queue counter (d_counters[0..8], and
// [16..21] for the kernels specialised to d = 3, 5, ..., 13).
static int launch_anneal(const xzzx_group *groups, const GroupWs *ws, int n_groups, AnnealMode mode,
                         uint64_t seed, int64_t unit_offset, int64_t units_override, uint32_t *d_counters,
                         hipStream_t stream)
{
    std::vector<int> rows_sel;
    std::vector<int> bytes_sel[7];
    std::vector<int> static_sel[kStaticMaxD + 1];
    std::vector<int> replay_cp;   // replays starting from checkpoints: one chain per wavefront
    int64_t total_syn = 0;
    for (int i = 0; i < n_groups; ++i) {
        if (groups[i].n_syn <= 0) continue;
        total_syn += groups[i].n_syn;
        const Plan &P = groups[i].plan->P;
        if (mode != AnnealMode::Replay && uses_static(groups[i], unit_offset)) static_sel[P.static_d].push_back(i);
        else if (mode == AnnealMode::Replay && checkpoints_of(groups[i]) > 0) replay_cp.push_back(i);
        else if (mode != AnnealMode::Replay && P.use_rows) rows_sel.push_back(i);
        else bytes_sel[log2_int(P.lanes)].push_back(i);
    }
    if (mode == AnnealMode::Replay) {
        // one chain per syndrome: enough wavefronts for 8 per CU
        std::vector<int> all;
        int C = kWave;
        for (int l = 0; l < 7; ++l)
            for (int i : bytes_sel[l]) {
                all.push_back(i);
                C = std::min(C, kWave / groups[i].plan->P.lanes);
            }
        const int64_t want = 8LL * device_cus();
        while (C > 1 && total_syn / C < want) C >>= 1;
        int rc = launch_set(groups, ws, all, false, kWave / C, mode, seed, unit_offset, units_override, d_counters,
                            stream);
        if (!rc)
            rc = launch_set(groups, ws, replay_cp, false, kWave, mode, seed, unit_offset, units_override,
                            d_counters + 2, stream);
        return rc;
    }
    int rc = launch_set(groups, ws, rows_sel, true, 1, mode, seed, unit_offset, units_override, d_counters, stream);
    for (int d = kStaticMinD; d <= kStaticMaxD && !rc; d += 2)
        rc = launch_set(groups, ws, static_sel[d], true, 1, mode, seed, unit_offset, units_override,
                        d_counters + 16 + (d - kStaticMinD) / 2, stream, d);
    for (int l = 0; l < 7 && !rc; ++l)
        rc = launch_set(groups, ws, bytes_sel[l], false, 1 << l, mode, seed, unit_offset, units_override,
                        d_counters + 1 + l, stream);
    return rc;
}

static int launch_reduce(const xzzx_group &g, const GroupWs &w, hipStream_t stream)
{
    if (g.n_syn == 0) return XZZX_OK;
    ReduceArgs A{};
    A.plan = g.plan->P.ddev;
    A.qcls = w.qcls;
    A.refs = w.refs;
    A.emin = w.emin;
    A.e_best = g.d_e_best;
    A.cls = g.d_cls;
    A.best_chain = w.best_chain;
    A.e_cls = g.d_e_cls;
    A.paper_recovery = g.d_paper_recovery;
    A.n_syn = g.n_syn;
    A.n_rep = g.n_rep;
    if (g.n_syn > 0x7FFFFFFF) { set_error("too many syndromes"); return XZZX_ERANGE; }
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)g.n_syn), dim3(kWave), 0, stream, A);
    return check_hip(hipGetLastError(), "k_reduce launch");
}

static int run_decode(const xzzx_group *groups, int n_groups, uint64_t greedy_seed, uint64_t anneal_seed,
                      int greedy_mode, int flags, void *d_workspace, size_t workspace_bytes,
                      hipStream_t stream, bool decode)
{
    int rc = validate_groups(groups, n_groups, decode);
    if (rc) return rc;
    if (decode && greedy_mode != XZZX_GREEDY_RANDOM && greedy_mode != XZZX_GREEDY_SAME &&
        greedy_mode != XZZX_GREEDY_BOUNDARY) {
        set_error("unknown greedy mode");
        return XZZX_EINVAL;
    }
    size_t need = 256;
    for (int i = 0; i < n_groups; ++i) need += group_ws_bytes(groups[i], decode);
    if (!d_workspace || workspace_bytes < need) { set_error("workspace too small"); return XZZX_ENOMEM; }
    uint8_t *p = static_cast<uint8_t *>(d_workspace);
    uint32_t *counter = reinterpret_cast<uint32_t *>(p);
    p += 256;
    std::vector<GroupWs> ws(n_groups);
    for (int i = 0; i < n_groups; ++i) ws[i] = carve_group(groups[i], decode, p);
    const int stage_bits = XZZX_FLAG_STAGE_GREEDY | XZZX_FLAG_STAGE_ANNEAL | XZZX_FLAG_STAGE_FINISH;
    const int stages = (flags & stage_bits) ? (flags & stage_bits) : stage_bits;
    for (int i = 0; i < n_groups; ++i) {
        const xzzx_group &g = groups[i];
        if (!decode || g.n_syn == 0 || !(stages & XZZX_FLAG_STAGE_GREEDY)) continue;
        rc = launch_greedy(g.plan->P, g.d_syn, g.d_uid, g.n_syn, g.n_rep, greedy_seed, greedy_mode, ws[i].refs,
                           ws[i].qraw, stream);
        if (!rc) rc = launch_qcls(ws[i].qraw, g.n_syn, g.n_rep, ws[i].qcls, stream);
        if (rc) return rc;
    }
    if (!(stages & XZZX_FLAG_STAGE_ANNEAL)) {
        // annealing skipped in this call
    } else if (flags & XZZX_FLAG_PLAIN) {
        // one launch per syndrome, grid = its own tasks, no persistence
        for (int i = 0; i < n_groups; ++i) {
            const xzzx_group &g = groups[i];
            for (int64_t s = 0; s < g.n_syn; ++s) {
                rc = launch_anneal(&g, &ws[i], 1, AnnealMode::Plain, anneal_seed, s * 4 * g.n_rep, 4 * g.n_rep, counter,
                                   stream);
                if (rc) return rc;
            }
        }
    } else {
        rc = launch_anneal(groups, ws.data(), n_groups, AnnealMode::Persistent, anneal_seed, 0, -1, counter, stream);
        if (rc) return rc;
    }
    if (!(stages & XZZX_FLAG_STAGE_FINISH)) return XZZX_OK;
    for (int i = 0; i < n_groups; ++i) {
        rc = launch_reduce(groups[i], ws[i], stream);
        if (rc) return rc;
    }
    return launch_anneal(groups, ws.data(), n_groups, AnnealMode::Replay, anneal_seed, 0, -1, counter + 8, stream);
}


// ---- serving launches (used by xzzx_server.cpp) ----
int serve_greedy(const Plan &P, const uint8_t *d_syn, int64_t syn_stride, const uint32_t *d_uid,
                 const int32_t *d_slot_map, int n, int n_rep, uint8_t *refs_base, int64_t refs_stride,
                 uint8_t *qraw_base, int64_t qraw_stride, uint64_t seed, int mode, hipStream_t stream)
{
    if (n <= 0) return XZZX_OK;
    GreedyArgs A{};
    A.plan = P.ddev;
    A.syn = d_syn;
    A.syn_stride = syn_stride;
    A.uid = d_uid;
    A.refs = refs_base;
    A.qraw = qraw_base;
    A.slot_map = d_slot_map;
    A.refs_stride = refs_stride;
    A.qraw_stride = qraw_stride;
    A.n_syn = n;
    A.n_rep = n_rep;
    A.mode = mode;
    A.seed_lo = (uint32_t)seed;
    A.seed_hi = (uint32_t)(seed >> 32);
    const int lds = greedy_lds(P, &A.max_nodes);
    hipLaunchKernelGGL(k_greedy, dim3((unsigned)(n * n_rep)), dim3(kWave), lds, stream, A);
    return check_hip(hipGetLastError(), "serving greedy launch");
}

int serve_slice(const ServeTask *d_rows, int n_rows, size_t lds_rows, const ServeTask *d_bytes, int n_bytes,
                size_t lds_bytes, uint64_t seed, hipStream_t stream)
{
    if (n_rows > 0)
        hipLaunchKernelGGL(k_serve_rows, dim3((unsigned)n_rows), dim3(kWave), lds_rows, stream, d_rows,
                           (uint32_t)seed, (uint32_t)(seed >> 32));
    if (n_bytes > 0)
        hipLaunchKernelGGL(k_serve_bytes, dim3((unsigned)n_bytes), dim3(kWave), lds_bytes, stream, d_bytes,
                           (uint32_t)seed, (uint32_t)(seed >> 32));
    return check_hip(hipGetLastError(), "serving slice launch");
}

int serve_finish(const ServeFinish *d_fin, const ServeTask *d_replay, int n, size_t lds_replay, uint64_t seed,
                 hipStream_t stream)
{
    if (n <= 0) return XZZX_OK;
    hipLaunchKernelGGL(k_serve_reduce, dim3((unsigned)n), dim3(kWave), 0, stream, d_fin);
    hipLaunchKernelGGL(k_serve_replay, dim3((unsigned)n), dim3(kWave), lds_replay, stream, d_replay,
                       (uint32_t)seed, (uint32_t)(seed >> 32));
    return check_hip(hipGetLastError(), "serving finish launch");
}

}  // namespace xzzx

using namespace xzzx;

extern "C" {

int xzzx_syndrome(const xzzx_plan *plan, const uint8_t *d_cfg, int64_t n, uint8_t *d_syn, void *stream)
{
    if (!plan || n < 0 || (n > 0 && (!d_cfg || !d_syn))) { set_error("bad syndrome arguments"); return XZZX_EINVAL; }
    if (n == 0) return XZZX_OK;
    const int64_t total = n * plan->P.lat.nstab;
    const int64_t blocks = (total + 255) / 256;
    if (blocks > 0x7FFFFFFF) { set_error("batch too large"); return XZZX_ERANGE; }
    hipLaunchKernelGGL(k_syndrome, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, plan->P.ddev, d_cfg, n, d_syn);
    return check_hip(hipGetLastError(), "k_syndrome launch");
}

int xzzx_greedy_init(const xzzx_plan *plan, const uint8_t *d_syn, const uint32_t *d_uid, int64_t n_syn,
                     int n_rep, uint64_t greedy_seed, int mode, uint8_t *d_refs, uint8_t *d_qcls, void *stream)
{
    if (!plan || n_syn < 0 || n_rep < 1) { set_error("bad greedy arguments"); return XZZX_EINVAL; }
    if (mode != XZZX_GREEDY_RANDOM && mode != XZZX_GREEDY_SAME && mode != XZZX_GREEDY_BOUNDARY) {
        set_error("unknown greedy mode");
        return XZZX_EINVAL;
    }
    if (n_syn == 0) return XZZX_OK;
    if (!d_syn || !d_uid || !d_refs || !d_qcls) { set_error("NULL buffer"); return XZZX_EINVAL; }
    // the raw symplectic bits land in d_qcls and are turned into classes in place
    int rc = launch_greedy(plan->P, d_syn, d_uid, n_syn, n_rep, greedy_seed, mode, d_refs, d_qcls, (hipStream_t)stream);
    if (rc) return rc;
    return launch_qcls(d_qcls, n_syn, n_rep, d_qcls, (hipStream_t)stream);
}

int xzzx_decode_workspace(const xzzx_group *groups, int n_groups, size_t *bytes)
{
    if (!groups || !bytes || n_groups < 1 || n_groups > kMaxGroups) { set_error("bad arguments"); return XZZX_EINVAL; }
    size_t need = 256;
    for (int i = 0; i < n_groups; ++i) {
        if (!groups[i].plan) { set_error("group without plan"); return XZZX_EINVAL; }
        need += group_ws_bytes(groups[i], true);
    }
    *bytes = need;
    return XZZX_OK;
}

int xzzx_decode(const xzzx_group *groups, int n_groups, uint64_t greedy_seed, uint64_t anneal_seed,
                int greedy_mode, int flags, void *d_workspace, size_t workspace_bytes, void *stream)
{
    return run_decode(groups, n_groups, greedy_seed, anneal_seed, greedy_mode, flags, d_workspace, workspace_bytes,
                      (hipStream_t)stream, true);
}

int xzzx_anneal(const xzzx_group *groups, int n_groups, uint64_t anneal_seed, int flags, void *d_workspace,
                size_t workspace_bytes, void *stream)
{
    return run_decode(groups, n_groups, 0, anneal_seed, XZZX_GREEDY_RANDOM, flags, d_workspace, workspace_bytes,
                      (hipStream_t)stream, false);
}

}  // extern "C"

struct xzzx_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

int xzzx_graph_create(const xzzx_group *groups, int n_groups, uint64_t greedy_seed, uint64_t anneal_seed,
                      int greedy_mode, int flags, void *d_workspace, size_t workspace_bytes, void *stream,
                      xzzx_graph **out)
{
    if (!out) { set_error("out is NULL"); return XZZX_EINVAL; }
    *out = nullptr;
    if (!stream) { set_error("graph capture needs a non-null stream"); return XZZX_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    int rc = check_hip(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (rc) return rc;
    const int drc = run_decode(groups, n_groups, greedy_seed, anneal_seed, greedy_mode, flags, d_workspace,
                               workspace_bytes, s, true);
    hipGraph_t g = nullptr;
    rc = check_hip(hipStreamEndCapture(s, &g), "hipStreamEndCapture");
    if (drc) {
        if (g) (void)hipGraphDestroy(g);
        return drc;
    }
    if (rc) return rc;
    auto *h = new xzzx_graph();
    h->graph = g;
    rc = check_hip(hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
    if (rc) {
        (void)hipGraphDestroy(g);
        delete h;
        return rc;
    }
    *out = h;
    return XZZX_OK;
}

int xzzx_graph_launch(xzzx_graph *graph, void *stream)
{
    if (!graph || !graph->exec) { set_error("graph is NULL"); return XZZX_EINVAL; }
    return check_hip(hipGraphLaunch(graph->exec, (hipStream_t)stream), "hipGraphLaunch");
}

void xzzx_graph_destroy(xzzx_graph *graph)
{
    if (!graph) return;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
}

}  // extern "C"
