// gfx950 kernels of the XZZX simulated-annealing decoder (those not
// specialised to a distance) and the device-side entry points of the C ABI.
//
//   k_syndrome     Eq. (2): syndrome of a batch of configurations.
//   k_greedy       Algs. 5-6: greedy matching per (syndrome, replica), both
//                  decoding-graph colours, paths XOR-ed into an LDS configuration.
//   k_qcls         Alg. 7: class Q_r of each reference relative to replica 0.
//   k_anneal<L>    Algs. 2-3 on byte-per-qubit states, 2^L lanes per chain
//                  (any lattice); k_anneal_rows: the generic packed-row kernel
//                  (rotated lattices, d <= 29).  Both are persistent: wavefronts
//                  pull tasks from an atomic queue spanning every syndrome group
//                  of the launch.  The packed-row kernels specialised to one
//                  distance (every odd d <= 31) are in xzzx_device.h /
//                  xzzx_static_*.hip.
//   k_replay<L>    re-runs each syndrome's best chain up to the phase of its
//                  minimum (from a checkpoint where the specialised kernel left
//                  one) and stores that state: the recovery.
//   k_reduce       Eqs. (18)-(21): per-coset minima, P*, best chain.
//   k_serve_*      the serving loop's slices, finish and result gather.
//
// The host half turns xzzx_group descriptions into launches: one persistent
// launch per kernel family and distance, run concurrently on side streams.
#include <hip/hip_runtime.h>

#include <utility>

#include <algorithm>
#include <functional>
#include <mutex>
#include <cstring>
#include <vector>

#include "xzzx_device.h"

namespace xzzx {

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
// Greedy matching (Algs. 5-6) -- one wavefront per (syndrome, replica), one
// colour per half wavefront or the colours in turn (see k_greedy).
//
// The sequential rule -- take the free pair of least (weight, key, pair id) --
// is evaluated as repeated mutual-best elimination: every free defect finds
// its least free partner, and pairs that are each other's least are matched.
// Under a strict total order the pair taken first by the sequential scan is
// always mutual-best, and removing matched defects never changes the order of
// the rest, so both procedures produce the same matching.  Paths follow the
// canonical tight-edge walk (smallest edge id) and are XOR-ed into the
// configuration with LDS atomics (paths may overlap).
// ---------------------------------------------------------------------------
// partners at the least weight a greedy scan lists before keying them, and
// partners whose interior distances a scan loads at once (the table is in
// HBM or L2: the loads of a batch overlap)
constexpr int kGreedyTies = 8;
constexpr int kGreedyBatch = 4;

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
    int rep_div;               // ladders: replica r draws the keys of replica r / rep_div (0 or 1: itself)
    int cache_entries;         // LDS words per colour for the pair weights (0: none)
    int64_t block0;            // (syndrome, replica) pair of workgroup 0 of this launch
};

__device__ __forceinline__ void xor_edge(uint32_t *cfgw, int eid)
{
    const int q = eid >> 1;
    const uint32_t code = (eid & 1) ? 2u : 1u;
    atomicXor(&cfgw[q >> 2], code << (8 * (q & 3)));
}

// Canonical walks.  Each step reads the node's four adjacency entries (in
// edge-id order) and their far ends' distances at once, then takes the first
// tight edge; the distance of the next node is known (dx - weight), so a step
// costs two dependent rounds of loads rather than one per entry tried.
__device__ void walk_interior(const PlanDev *pl, int g, int u, int v, uint32_t *cfgw)
{
    const int n = pl->ncol[g];
    const int32_t *du = pl->dint[g] + (size_t)u * n;
    const int4 *adj = pl->adj[g];
    int x = v;
    int32_t dx = du[x];
    for (int step = 0; step < n && x != u; ++step) {
        int4 e[4];
        int32_t de[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) e[s] = adj[4 * x + s];
#pragma unroll
        for (int s = 0; s < 4; ++s) de[s] = (e[s].x >= 0 && e[s].y >= 0) ? du[e[s].y] : -1;
        int nxt = -1;
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if (nxt < 0 && e[s].x >= 0 && e[s].y >= 0 && de[s] + e[s].z == dx) {
                xor_edge(cfgw, e[s].x);
                nxt = e[s].y;
                dx = de[s];
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
    int32_t dx = db[x];
    for (int step = 0; step <= n; ++step) {
        int4 e[4];
        int32_t de[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) e[s] = adj[4 * x + s];
#pragma unroll
        for (int s = 0; s < 4; ++s) de[s] = (e[s].x >= 0 && e[s].y >= 0) ? db[e[s].y] : -1;
        // the first tight entry in edge-id order: a boundary half-edge ends the walk
        int nxt = -1;
        bool done = false;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (done || nxt >= 0 || e[s].x < 0) continue;
            if (e[s].y < 0) {
                if (e[s].z == dx) { xor_edge(cfgw, e[s].x); done = true; }
            } else if (de[s] + e[s].z == dx) {
                xor_edge(cfgw, e[s].x);
                nxt = e[s].y;
                dx = de[s];
            }
        }
        if (done || nxt < 0) return;
        x = nxt;
    }
}

// SPLIT: the two decoding-graph colours are independent matchings, so each
// half of the wavefront (32 lanes) runs one, and both XOR their paths into the
// shared configuration -- twice the lanes at work where a colour has no more
// than a few dozen defects.  Otherwise the whole wavefront runs the colours one
// after the other.  The kernel waits on memory most of the time, so the split
// form is held to eight wavefronts per SIMD (64 VGPRs; at its natural 68 it
// ran seven, and the d = 11 and planar d = 9 greedy stages took 4-5 % longer).
template <bool SPLIT>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(SPLIT ? 8 : 1, 8))) void k_greedy(GreedyArgs A)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const PlanDev *pl = A.plan;
    const int lane = threadIdx.x;
    const int nq = pl->nq;
    const int64_t sr = A.block0 + blockIdx.x;
    const int64_t s = sr / A.n_rep;
    const uint32_t r = (uint32_t)(sr - s * A.n_rep);
    const uint32_t rkey = A.rep_div > 1 ? r / (uint32_t)A.rep_div : r;
    const uint32_t uid = A.uid[s];
    const int nwords = (nq + 3) / 4;
    constexpr int kHalf = SPLIT ? kWave / 2 : kWave;   // lanes per colour
    const int hl = lane % kHalf;
    const int stride = A.max_nodes + 1;
    uint32_t *cfgw = reinterpret_cast<uint32_t *>(smem);
    // per colour: D, best, pairs, dbD, the free flags and the list of free
    // defects (the colours in turn share one set)
    constexpr int kSets = SPLIT ? 2 : 1;
    int16_t *cands = reinterpret_cast<int16_t *>(reinterpret_cast<int32_t *>(smem + 4 * nwords) + kSets * 4 * stride);
    // the free flags (bytes), then the free lists (int16, 2-byte aligned),
    // then the pair-weight cache, 16-byte aligned
    const uint32_t flags_off = 4u * nwords + kSets * 4 * 4 * stride + 2 * kWave * kGreedyTies;
    const uint32_t list_off = (flags_off + kSets * stride + 1u) & ~1u;
    const uint32_t cache_off = (list_off + kSets * 2 * stride + 15u) & ~15u;
    __shared__ int s_count[2];

    for (int i = lane; i < nwords; i += kWave) cfgw[i] = 0;
    if (lane == 0) { s_count[0] = 0; s_count[1] = 0; }
    const uint8_t *sy = A.syn + s * A.syn_stride;
    const int n_both = max(pl->ncol[0], pl->ncol[1]);
    for (int gg = 0; gg < (SPLIT ? 1 : 2); ++gg) {
        const int g = SPLIT ? lane / kHalf : gg;
        const int set = SPLIT ? g : 0;
        int32_t *D = reinterpret_cast<int32_t *>(smem + 4 * nwords) + set * 4 * stride;
        int32_t *best = D + stride;
        int32_t *pairs = best + stride;
        int32_t *dbD = pairs + stride;   // boundary distance of each defect
        uint8_t *freef = smem + flags_off + set * stride;
        int16_t *fl = reinterpret_cast<int16_t *>(smem + list_off) + set * stride;
        const int n = pl->ncol[g];
        const int32_t *cf = pl->col_face[g];
        const int32_t *dint = pl->dint[g];
        const int32_t *db = pl->db[g];
        // defects of this colour, ascending node index
        int nd = 0;
        for (int base = 0; base < (SPLIT ? n_both : n); base += kHalf) {
            const int v = base + hl;
            const bool flag = v < n && sy[cf[v]];
            const uint64_t mask = SPLIT ? ((__ballot(flag) >> (g * kHalf)) & 0xFFFFFFFFull) : __ballot(flag);
            const int pos = nd + __popcll(mask & ((1ull << hl) - 1ull));
            if (flag) D[pos] = v;
            nd += __popcll(mask);
        }
        __syncthreads();
        if (A.mode == XZZX_GREEDY_BOUNDARY) {
            for (int i = hl; i < nd; i += kHalf) walk_boundary(pl, g, D[i], cfgw);
        } else {
            const int na = nd + (nd & 1);   // odd count: the virtual boundary joins as node nd
            for (int i = hl; i < na; i += kHalf) freef[i] = 1;
            for (int i = hl; i < nd; i += kHalf) dbD[i] = db[D[i]];
            __syncthreads();
            int nfree = na;
            const bool randomized = A.mode == XZZX_GREEDY_RANDOM;
            // a pair (i, j) weighs the interior distance or the two boundary
            // distances, whichever is less; a pair with the virtual node (an
            // odd count) weighs the real defect's boundary distance
            auto weight_of_pair = [&](int i, int j, int32_t dj) -> uint32_t {
                return i == nd ? (uint32_t)dbD[j] : j == nd ? (uint32_t)dbD[i] : (uint32_t)min(dj, dbD[i] + dbD[j]);
            };
            // every pair weight in LDS when the defects fit the cache (rows of
            // an odd stride: the lanes' reads of one column fall in distinct
            // banks), so the rounds after the first scan LDS, not the table in
            // L2; the weights are the same either way
            uint32_t *wc = reinterpret_cast<uint32_t *>(smem + cache_off) + set * A.cache_entries;
            const int rs = na | 1;
            const bool cached = (int64_t)na * rs <= (int64_t)A.cache_entries;
            if (cached) {
                for (int i = hl; i < na; i += kHalf) {
                    const int32_t *drow = dint + (size_t)(i == nd ? 0 : D[i]) * n;
                    for (int j0 = 0; j0 < na; j0 += kGreedyBatch) {
                        int32_t dv[kGreedyBatch];
#pragma unroll
                        for (int k = 0; k < kGreedyBatch; ++k) dv[k] = drow[j0 + k < nd ? D[j0 + k] : 0];
#pragma unroll
                        for (int k = 0; k < kGreedyBatch; ++k)
                            if (j0 + k < na) wc[i * rs + j0 + k] = weight_of_pair(i, j0 + k, dv[k]);
                    }
                }
            }
            __syncthreads();
            // every round matches at least the least free pair, so na/2 rounds
            // suffice (rounds continue while either half has work).  Free
            // defects only leave, so a defect whose least partner is still free
            // keeps it; only the others search again.
            const int na_all = SPLIT ? max(__shfl(na, 0, kWave), __shfl(na, kHalf, kWave)) : na;
            for (int round = 0; __ballot(nfree > 0 && round <= na / 2) != 0; ++round) {
                // the free defects of this colour, ascending: the defects and
                // the partners the round scans come from this list, so a late
                // round skips the ones already matched (the same candidates in
                // the same order; the greedy stage at d = 31 took half the
                // time)
                int nfl = 0;
                for (int base = 0; base < na_all; base += kHalf) {
                    const int v = base + hl;
                    const bool flag = v < na && freef[v];
                    const uint64_t mask = SPLIT ? ((__ballot(flag) >> (g * kHalf)) & 0xFFFFFFFFull) : __ballot(flag);
                    const int pos = nfl + __popcll(mask & ((1ull << hl) - 1ull));
                    if (flag) fl[pos] = (int16_t)v;
                    nfl += __popcll(mask);
                }
                __syncthreads();
                for (int t = hl; t < nfl; t += kHalf) {
                    const int i = fl[t];
                    if (round > 0 && best[i] >= 0 && freef[best[i]]) continue;
                    // least (w, key, id) over free partners j, in two passes: the
                    // least weight and the partners at it (in ascending j, so
                    // ascending pair id), then keys for those partners only -- a
                    // single scan that drew a key on every tie so far made the
                    // wavefront draw one for nearly every partner.  The interior
                    // distances of a batch of partners are loaded before any is used.
                    const bool iv = i == nd;   // the virtual boundary node
                    const int32_t *drow = dint + (size_t)(iv ? 0 : D[i]) * n;
                    const uint32_t *wrow = wc + i * rs;
                    int16_t *cand = cands + lane * kGreedyTies;
                    auto weight = [&](int j, int32_t dj) -> uint32_t {
                        return cached ? wrow[j] : weight_of_pair(i, j, dj);
                    };
                    uint32_t bw = 0xFFFFFFFFu;
                    int nt = 0;   // partners at weight bw
                    for (int t0 = 0; t0 < nfl; t0 += kGreedyBatch) {
                        int32_t dv[kGreedyBatch];
                        int jj[kGreedyBatch];
#pragma unroll
                        for (int k = 0; k < kGreedyBatch; ++k) jj[k] = t0 + k < nfl ? fl[t0 + k] : na;
#pragma unroll
                        for (int k = 0; k < kGreedyBatch; ++k)
                            dv[k] = cached ? 0 : drow[jj[k] < nd ? D[jj[k]] : 0];
#pragma unroll
                        for (int k = 0; k < kGreedyBatch; ++k) {
                            const int j = jj[k];
                            if (j >= na || j == i) continue;
                            const uint32_t w = weight(j, dv[k]);
                            if (w > bw) continue;
                            if (w < bw) { bw = w; nt = 0; }
                            if (nt < kGreedyTies) cand[nt] = (int16_t)j;
                            ++nt;
                        }
                    }
                    int bj = nt > 0 ? cand[0] : -1;
                    if (randomized && nt > 1) {
                        auto pair_id = [&](int j) { return (uint32_t)(min(i, j) * na + max(i, j)); };
                        auto pair_key = [&](uint32_t id) {
                            return philox4x32_10(make_uint4(uid, rkey, 0x100u + (uint32_t)g, id), A.seed_lo, A.seed_hi).x;
                        };
                        uint32_t bid = pair_id(bj), bk = pair_key(bid);
                        if (nt <= kGreedyTies) {
                            for (int t = 1; t < nt; ++t) {
                                const int j = cand[t];
                                const uint32_t id = pair_id(j), key = pair_key(id);
                                if (key < bk) { bk = key; bid = id; bj = j; }   // ids ascend: ties keep the first
                            }
                        } else {
                            // more ties than the list holds: scan again
                            for (int j = bj + 1; j < na; ++j) {
                                if (j == i || !freef[j]) continue;
                                const int32_t dj = (!cached && !iv && j < nd) ? drow[D[j]] : 0;
                                if (weight(j, dj) != bw) continue;
                                const uint32_t id = pair_id(j), key = pair_key(id);
                                if (key < bk) { bk = key; bid = id; bj = j; }
                            }
                        }
                    }
                    best[i] = bj;
                }
                __syncthreads();
                for (int t = hl; t < nfl; t += kHalf) {
                    const int i = fl[t];
                    const int j = best[i];
                    if (j > i && best[j] == i) {
                        const int p = atomicAdd(&s_count[g], 1);
                        pairs[p] = i | (j << 16);
                    }
                }
                __syncthreads();
                const int np = s_count[g];
                for (int p = hl; p < np; p += kHalf) {
                    freef[pairs[p] & 0xFFFF] = 0;
                    freef[pairs[p] >> 16] = 0;
                }
                __syncthreads();
                nfree = na - 2 * np;
            }
            const int np = s_count[g];
            for (int p = hl; p < np; p += kHalf) {
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

// Caller-supplied references (the anneal-only entry point), one wavefront per
// (syndrome, replica): the raw symplectic products with L_Z and L_X, as the
// greedy kernel writes them, and, when syndromes are given, whether the
// reference has syndrome S (Alg. 7 requires a configuration with boundary S;
// Eq. (2)).  A mismatch sets *bad.
__global__ __launch_bounds__(kWave) void k_ref_check(const PlanDev *__restrict__ pl, const uint8_t *__restrict__ refs,
                                                     const uint8_t *__restrict__ syn, int n_rep, int64_t block0,
                                                     uint8_t *__restrict__ qraw, uint32_t *bad)
{
    const int nq = pl->nq, nstab = pl->nstab, lane = threadIdx.x;
    const int64_t sr = block0 + blockIdx.x;
    const uint8_t *c = refs + sr * nq;
    uint32_t vz = 0, vx = 0;
    for (int q = lane; q < nq; q += kWave) {
        const uint32_t v = c[q], z = pl->lz[q], x = pl->lx[q];
        vz ^= (((v >> 1) & z) ^ (v & (z >> 1))) & 1;
        vx ^= (((v >> 1) & x) ^ (v & (x >> 1))) & 1;
    }
    const int az = __popcll(__ballot(vz)) & 1;
    const int ax = __popcll(__ballot(vx)) & 1;
    if (lane == 0) qraw[sr] = (uint8_t)(az | (ax << 1));
    if (!syn) return;
    const uint8_t *S = syn + (sr / n_rep) * nstab;
    uint32_t diff = 0;
    for (int f = lane; f < nstab; f += kWave) {
        const Desc d = pl->face_desc[f];
        const int q[4] = {(int)(d.x & 0xFFFF), (int)(d.x >> 16), (int)(d.y & 0xFFFF), (int)((d.y >> 16) & 0x7FF)};
        uint32_t bit = 0;
        if (q[0] < nq) bit ^= c[q[0]] & 1;
        if (q[1] < nq) bit ^= (c[q[1]] >> 1) & 1;
        if (q[2] < nq) bit ^= (c[q[2]] >> 1) & 1;
        if (q[3] < nq) bit ^= c[q[3]] & 1;
        diff |= bit ^ (S[f] & 1u);
    }
    if (__ballot(diff) && lane == 0) atomicOr(bad, 1u);
}

template <int LOGG>
__global__ __launch_bounds__(kWave) void k_anneal(AnnealArgs A) { batch_kernel_body<0, false, LOGG, false>(A); }
template <int LOGG>
__global__ __launch_bounds__(kWave) void k_replay(AnnealArgs A) { batch_kernel_body<0, false, LOGG, true>(A); }
template <int LOGG>
__global__ __launch_bounds__(kWave) void k_anneal_plain(AnnealArgs A) { batch_kernel_body<2, false, LOGG, false>(A); }
__global__ __launch_bounds__(kWave) void k_anneal_site(AnnealArgs A) { site_kernel_body<0>(A); }
__global__ __launch_bounds__(kWave) void k_anneal_site_plain(AnnealArgs A) { site_kernel_body<2>(A); }

// Random-site order: each syndrome's recovery is its best chain's state kept
// at that chain's first E_min (packed words [word][chain]); one thread per
// (syndrome, qubit).
__global__ void k_site_recovery(const uint32_t *__restrict__ snap, int64_t n_chains,
                                const int32_t *__restrict__ best_chain, int n_rep, int nq, int64_t n_syn,
                                uint8_t *__restrict__ recovery)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_syn * nq) return;
    const int64_t s = idx / nq;
    const int q = (int)(idx - s * nq);
    const int64_t ci = s * 4 * n_rep + best_chain[s];
    recovery[idx] = (uint8_t)((snap[(int64_t)(q >> 4) * n_chains + ci] >> (2 * (q & 15))) & 3u);
}

// Planar kernel specialised to d: the same from its rows, chain-major with
// `words` words per chain (word Y * nw + c / 16 holds the qubit at row Y,
// column c), one thread per (syndrome, qubit).
__global__ void k_rows_recovery(const uint32_t *__restrict__ snap, int words,
                                const int32_t *__restrict__ best_chain, int n_rep, int nq, int64_t n_syn,
                                const PlanDev *__restrict__ pl, int nw, uint8_t *__restrict__ recovery)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_syn * nq) return;
    const int64_t s = idx / nq;
    const int q = (int)(idx - s * nq);
    const int64_t ci = s * 4 * n_rep + best_chain[s];
    const uint32_t p = pl->qpos[q];
    const uint32_t word = snap[ci * words + (int64_t)((p >> 8) * nw + ((p & 0xFFu) >> 4))];
    recovery[idx] = (uint8_t)((word >> (2 * (p & 15u))) & 3u);
}
// Rotated ladder kernel specialised to d: the same from its rows,
// chain-major with `words` words per chain (word y * nw + x / 16 holds the
// qubit at row y, column x), one thread per (syndrome, qubit).
__global__ void k_static_recovery(const uint32_t *__restrict__ snap, int words,
                                  const int32_t *__restrict__ best_chain, int n_rep, int d, int64_t n_syn, int nw,
                                  uint8_t *__restrict__ recovery)
{
    const int nq = d * d;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_syn * nq) return;
    const int64_t s = idx / nq;
    const int q = (int)(idx - s * nq);
    const int y = q / d, x = q - y * d;
    const int64_t ci = s * 4 * n_rep + best_chain[s];
    const uint32_t word = snap[ci * words + (int64_t)(y * nw + (x >> 4))];
    recovery[idx] = (uint8_t)((word >> (2 * (x & 15))) & 3u);
}
__global__ __launch_bounds__(kWave) void k_anneal_rows(AnnealArgs A) { batch_kernel_body<0, true, 0, false>(A); }
__global__ __launch_bounds__(kWave) void k_anneal_rows_plain(AnnealArgs A) { batch_kernel_body<2, true, 0, false>(A); }

static AnnealKernel static_rows_kernel(int d, bool plain)
{
#define XZZX_TRY_PART(P) \
    if (AnnealKernel k = static_rows_kernel_##P(d, plain)) return k;
    XZZX_STATIC_PARTS(XZZX_TRY_PART)
#undef XZZX_TRY_PART
    return nullptr;
}

// serving kernel of the specialised class holding d (NULL outside [3, 31])
static ServeKernel static_serve_kernel(int d)
{
    if (d < kStaticMinD || d > kStaticMaxD) return nullptr;
    switch (serve_class_max(d)) {
    case 9: return serve_class_kernel_9();
    case 15: return serve_class_kernel_15();
    case 21: return serve_class_kernel_21();
    case 25: return serve_class_kernel_25();
    case 29: return serve_class_kernel_29();
    default: return serve_class_kernel_31();
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

// Before a slice: every task resuming at t_begin > 0 copies the stored state
// of each of its chains into the chain's buffer that its replay entry does
// not name (the range's start state, for a later replay).  One workgroup per
// task, bytes of the task's chains spread over the lanes.
__global__ __launch_bounds__(256) void k_serve_stash(const ServeTask *tasks)
{
    const ServeTask &T = tasks[blockIdx.x];
    if (T.t_begin == 0 || !T.cpm) return;
    const int nq = T.plan->nq;
    const int64_t nc = 4 * (int64_t)T.n_rep;
    const int64_t total = (int64_t)T.nchains * nq;
    for (int64_t i = threadIdx.x; i < total; i += blockDim.x) {
        const int64_t k = i / nq;
        const int64_t c = T.chain0 + k, q = i - k * nq;
        const int64_t b = kept_scratch(T.cpm[c]);
        T.cp[(b * nc + c) * nq + q] = T.states[c * nq + q];
    }
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
// Results and recoveries of the finished requests, packed for one copy to the host.
__global__ __launch_bounds__(kWave) void k_serve_gather(const ServeFinish *fin)
{
    const ServeFinish &F = fin[blockIdx.x];
    const int lane = threadIdx.x;
    if (lane < 8) reinterpret_cast<int32_t *>(F.out)[lane] = F.result[lane];
    for (int q = lane; q < F.nq; q += kWave) F.out[32 + q] = F.recovery[q];
}

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
// A launch addresses at most 2^32 - 1 work-items (larger grids wrap
// silently), i.e. this many wavefronts of 64.
constexpr int64_t kMaxLaunchItems = 0xFFFFFFFFll;
constexpr int64_t kMaxLaunchWaves = kMaxLaunchItems / kWave;

static int check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return XZZX_OK;
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return XZZX_EDEVICE;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// One colour per half wavefront where a colour has at most 128 nodes (rotated
// d <= 15: few enough defects that 32 lanes take them in one or two turns);
// the whole wavefront per colour on larger lattices.
static bool greedy_split(const Plan &P) { return std::max(P.hdev.ncol[0], P.hdev.ncol[1]) <= 128; }

// LDS of a greedy workgroup: the configuration, per colour set D, best,
// pairs, dbD, the free flags and the free list (one set per colour when the
// halves of the wavefront match the colours at once, else one), the tie
// lists, and, with `cache` (launches of few wavefronts, where latency matters
// more than occupancy), the pair-weight cache of each set: 16 KiB per colour
// when the colours run side by side (up to 63 defects), 48 KiB otherwise (up
// to 109).
static int greedy_lds(const Plan &P, bool cache, GreedyArgs *A)
{
    const int mn = std::max(P.hdev.ncol[0], P.hdev.ncol[1]);
    A->max_nodes = mn;
    const int sets = greedy_split(P) ? 2 : 1;
    const int flags = 4 * ((P.lat.nq + 3) / 4) + sets * 4 * 4 * (mn + 1) + 2 * kWave * kGreedyTies;
    const int base = ((flags + sets * (mn + 1) + 1) & ~1) + sets * 2 * (mn + 1);
    A->cache_entries = cache ? (sets == 2 ? 4096 : 12288) : 0;
    return ((base + 15) & ~15) + sets * 4 * A->cache_entries + 16;
}

// launches of at most this many (syndrome, replica) wavefronts cache the pair
// weights in LDS (larger ones keep the occupancy instead: a serving slice
// admitting thousands of requests ran its greedy launches 20 % slower with
// the cache)
constexpr int64_t kGreedyCacheWaves = 2048;

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
    A.rep_div = P.ladder_k;
    A.syn_stride = P.lat.nstab;
    A.seed_lo = (uint32_t)seed;
    A.seed_hi = (uint32_t)(seed >> 32);
    // one launch addresses fewer than 2^32 work-items: the (syndrome, replica)
    // pairs go in chunks of at most that many wavefronts
    const int64_t blocks = n_syn * n_rep;
    const int lds = greedy_lds(P, blocks <= kGreedyCacheWaves, &A);
    for (int64_t b0 = 0; b0 < blocks; b0 += kMaxLaunchWaves) {
        A.block0 = b0;
        const int64_t nb = std::min<int64_t>(kMaxLaunchWaves, blocks - b0);
        hipLaunchKernelGGL(greedy_split(P) ? k_greedy<true> : k_greedy<false>, dim3((unsigned)nb), dim3(kWave), lds,
                           stream, A);
        const int rc = check_hip(hipGetLastError(), "k_greedy launch");
        if (rc) return rc;
    }
    return XZZX_OK;
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
    uint32_t *min_snap;    // random-site and planar specialised groups: each chain's state at its first E_min
};

// Replica exchange on the packed-row kernels specialised to d: the distance
// when the group's ladders run there (rotated: d <= kLadderRowsMaxD and every
// 64-chain task inside one syndrome; planar: d <= 15), else 0.  Depends on
// the plan and n_rep only, so every stage of a decode agrees.
static int ladder_rows_d(const xzzx_group &g)
{
    const Plan &P = g.plan->P;
    if (!P.ladder_k || !P.use_rows || P.order != XZZX_ORDER_COLOUR) return 0;
    if (P.static_d && P.static_d <= kLadderRowsMaxD && (4 * g.n_rep) % kWave == 0) return P.static_d;
    return 0;
}

static int ladder_planar_d(const xzzx_group &g)
{
    const Plan &P = g.plan->P;
    if (!P.ladder_k || !P.use_rows || P.order != XZZX_ORDER_COLOUR) return 0;
    return P.planar_d;
}

// Words per chain of the state kept at E_min: random-site chains and the
// generic ladder kernel (packed, the position nq scratch), the planar kernels
// specialised to d and the rotated ladder kernels specialised to d (their
// rows); 0 for other groups.  A plan's kernel must not change between the
// stages of one decode.
static int64_t min_snap_words(const xzzx_group &g)
{
    const Plan &P = g.plan->P;
    if (ladder_rows_d(g)) return ladder_rows_state_words(ladder_rows_d(g));
    if (ladder_planar_d(g)) return planar_state_words(ladder_planar_d(g));
    if (P.order == XZZX_ORDER_RANDOM_SITE || P.ladder_k) return P.lat.nq / 16 + 1;
    if (P.use_rows && P.planar_d) return planar_state_words(P.planar_d);
    return 0;
}

// A group runs on the packed-row kernel specialised to its distance when the
// plan allows it and every 64-chain task lies inside one syndrome.
static bool uses_static(const xzzx_group &g, int64_t unit_offset)
{
    const Plan &P = g.plan->P;
    return P.order == XZZX_ORDER_COLOUR && !P.ladder_k && P.use_rows && P.static_d && (4 * g.n_rep) % kWave == 0 &&
           unit_offset % kWave == 0;
}

// Sweeps between the checkpoints of a plan: kCheckpointEvery, or the least
// interval that leaves at most kMaxCheckpoints before the last sweep.
static int checkpoint_interval(const Plan &P)
{
    const int spread = (P.n_sweeps - 1 + kMaxCheckpoints - 1) / kMaxCheckpoints;
    return std::max(kCheckpointEvery, spread);
}

// Checkpoints a specialised group keeps: the states at the start of sweeps
// c, 2c, ... before the last sweep, for c = checkpoint_interval.
static int checkpoints_of(const xzzx_group &g)
{
    if (!uses_static(g, 0) || g.plan->P.n_sweeps <= 0) return 0;
    return (g.plan->P.n_sweeps - 1) / checkpoint_interval(g.plan->P);
}

static size_t group_ws_bytes(const xzzx_group &g, bool decode)
{
    const Plan &P = g.plan->P;
    const size_t nq = P.lat.nq, ns = (size_t)g.n_syn, R = (size_t)g.n_rep, nc = 4 * R * ns;
    size_t b = 0;
    if (decode && !g.d_refs) b += align256(ns * R * nq);
    b += align256(ns * R);                                  // qraw
    if (!g.d_qcls) b += align256(ns * R);
    if (!g.d_chain_emin) b += align256(nc * 4);
    if (!g.d_chain_stop) b += align256(nc * 4);
    if (!g.d_chain_e) b += align256(nc * 4);
    if (!g.d_best_chain) b += align256(ns * 4);
    b += align256((size_t)checkpoints_of(g) * P.lat.d * P.static_words * nc * 4);
    b += align256((size_t)min_snap_words(g) * nc * 4);
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
    w.qcls = g.d_qcls ? g.d_qcls : take(ns * R);
    w.emin = g.d_chain_emin ? g.d_chain_emin : reinterpret_cast<int32_t *>(take(nc * 4));
    w.stop = g.d_chain_stop ? g.d_chain_stop : reinterpret_cast<int32_t *>(take(nc * 4));
    w.efin = g.d_chain_e ? g.d_chain_e : reinterpret_cast<int32_t *>(take(nc * 4));
    w.best_chain = g.d_best_chain ? g.d_best_chain : reinterpret_cast<int32_t *>(take(ns * 4));
    const int ncp = checkpoints_of(g);
    w.cp_rows = ncp ? reinterpret_cast<uint32_t *>(take((size_t)ncp * P.lat.d * P.static_words * nc * 4)) : nullptr;
    w.min_snap = min_snap_words(g) ? reinterpret_cast<uint32_t *>(take((size_t)min_snap_words(g) * nc * 4)) : nullptr;
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
        if (g.plan->P.ladder_k && g.n_rep % g.plan->P.ladder_k) { set_error("n_rep must be a multiple of the ladder's levels"); return XZZX_EINVAL; }
        if (g.plan->P.device != dev) { set_error("plan was created on another device"); return XZZX_EINVAL; }
        if (g.n_syn == 0) continue;
        if (!g.d_uid || !g.d_e_best || !g.d_cls || !g.d_recovery) { set_error("missing required group buffer"); return XZZX_EINVAL; }
        if (decode && !g.d_syn) { set_error("decode needs d_syn"); return XZZX_EINVAL; }
        if (!decode && !g.d_refs) { set_error("anneal needs d_refs"); return XZZX_EINVAL; }
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
                      uint32_t *d_counter, hipStream_t stream, int static_d = 0, bool site = false,
                      int planar_d = 0, bool ladder = false)
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
        G.cp_every = cp ? checkpoint_interval(P) : 0;
        G.n_chains = g.n_syn * 4 * g.n_rep;
        G.min_snap = (site || planar_d || ladder) ? ws[i].min_snap : nullptr;
        G.unit_offset = unit_offset;
        const int64_t units = units_of(i);
        G.n_units = units;
        G.task_begin = (int64_t)tasks;
        const int C = kWave / lanes;
        tasks += (uint64_t)((units + C - 1) / C);
        lds = std::max(lds, (ladder && (static_d || planar_d))
                                ? 16 * (size_t)P.ladder_k * P.nranks()
                            : (static_d || planar_d) ? (size_t)0
                            : ladder ? P.lds_bytes_ladder()
                            : site   ? P.lds_bytes_site()
                            : rows   ? P.lds_bytes_rows()
                                     : P.lds_bytes_anneal(lanes));
    }
    if (ng == 0 || tasks == 0) return XZZX_OK;
    if (tasks >= 0xFFFFFFF0ull) { set_error("too many anneal tasks in one launch"); return XZZX_ERANGE; }
    A.n_groups = ng;
    A.n_tasks = (uint32_t)tasks;
    if (lds > 65536) { set_error("LDS demand above 64 KiB"); return XZZX_ERANGE; }
    if (mode == AnnealMode::Plain) {
        if (ladder && static_d)
            hipLaunchKernelGGL(ladder_rows_kernel(static_d, true), dim3((unsigned)tasks), dim3(kWave), lds, stream, A);
        else if (ladder && planar_d)
            hipLaunchKernelGGL(ladder_planar_kernel(planar_d, true), dim3((unsigned)tasks), dim3(kWave), lds, stream, A);
        else if (ladder)
            hipLaunchKernelGGL(ladder_kernel(true), dim3((unsigned)tasks), dim3(kWave), lds, stream, A);
        else if (site)
            hipLaunchKernelGGL(k_anneal_site_plain, dim3((unsigned)tasks), dim3(kWave), lds, stream, A);
        else if (planar_d)
            hipLaunchKernelGGL(planar_rows_kernel(planar_d, true), dim3((unsigned)tasks), dim3(kWave), 0, stream, A);
        else if (static_d)
            hipLaunchKernelGGL(static_rows_kernel(static_d, true), dim3((unsigned)tasks), dim3(kWave), 0, stream, A);
        else if (rows)
            hipLaunchKernelGGL(k_anneal_rows_plain, dim3((unsigned)tasks), dim3(kWave), lds, stream, A);
        else
            hipLaunchKernelGGL(bytes_kernel(2, lg), dim3((unsigned)tasks), dim3(kWave), lds, stream, A);
        return check_hip(hipGetLastError(), "plain anneal launch");
    }
    const AnnealKernel kern = (ladder && static_d) ? ladder_rows_kernel(static_d, false)
                              : (ladder && planar_d) ? ladder_planar_kernel(planar_d, false)
                              : ladder     ? ladder_kernel(false)
                              : site     ? k_anneal_site
                              : planar_d ? planar_rows_kernel(planar_d, false)
                              : static_d ? static_rows_kernel(static_d, false)
                              : rows     ? k_anneal_rows
                                         : bytes_kernel(replay ? 1 : 0, lg);
    unsigned grid = 0;
    int rc = anneal_grid((const void *)kern, lds, A.n_tasks, &grid);
    if (rc) return rc;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, stream, d_counter, 1);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWave), lds, stream, A);
    return check_hip(hipGetLastError(), "anneal launch");
}

// Side streams (default priority) and reusable events for running the
// independent launches of one call concurrently.  Each (device, caller stream)
// pair has a set of its own, created on first use and kept until the process
// ends, so calls on different streams -- among them a graph capture on one
// stream and a serving loop on another -- never share a side stream; calls on
// one caller stream hold the set's lock while they fork and join.  Past
// kMaxSideSets sets, calls run their launches one after another on the caller
// stream instead (same results).
constexpr int kSideStreams = 3;
constexpr int kMaxSideSets = 256;

struct SideSet {
    std::mutex mu;
    hipStream_t side[kSideStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kSideStreams] = {};
};

// The set of `caller` on the current device, nullptr when the table is full;
// an error status if a stream or event cannot be created.
static int side_set(hipStream_t caller, SideSet **out)
{
    static std::mutex mu;
    static std::vector<std::pair<std::pair<int, hipStream_t>, SideSet *>> sets;   // never freed
    *out = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { set_error("hipGetDevice failed"); return XZZX_EDEVICE; }
    const std::pair<int, hipStream_t> key(dev, caller);
    std::lock_guard<std::mutex> lk(mu);
    for (auto &e : sets)
        if (e.first == key) { *out = e.second; return XZZX_OK; }
    if ((int)sets.size() >= kMaxSideSets) return XZZX_OK;
    auto *S = new SideSet();
    bool ok = hipEventCreateWithFlags(&S->fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < kSideStreams && ok; ++i)
        ok = hipStreamCreateWithFlags(&S->side[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&S->join[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        for (int i = 0; i < kSideStreams; ++i) {
            if (S->side[i]) (void)hipStreamDestroy(S->side[i]);
            if (S->join[i]) (void)hipEventDestroy(S->join[i]);
        }
        if (S->fork) (void)hipEventDestroy(S->fork);
        delete S;
        set_error("side stream or event creation failed");
        return XZZX_EDEVICE;
    }
    sets.emplace_back(key, S);
    *out = S;
    return XZZX_OK;
}

// Runs launch(i, stream_i) for i < n: launch 0 on `stream`, the others on the
// caller's side streams, which wait for `stream`'s prior work; `stream` then
// waits for all.  Works under hipGraph capture (the events become graph
// dependencies).  serial: every launch on `stream`, in order (no side
// streams or events are created or used).
template <typename F>
static int fork_join(hipStream_t stream, int n, F launch, bool serial = false)
{
    if (serial) {
        int rc = XZZX_OK;
        for (int i = 0; i < n && !rc; ++i) rc = launch(i, stream);
        return rc;
    }
    if (n <= 1) return n ? launch(0, stream) : XZZX_OK;
    SideSet *S = nullptr;
    int rc = side_set(stream, &S);
    if (rc) return rc;
    if (!S) {
        for (int i = 0; i < n && !rc; ++i) rc = launch(i, stream);
        return rc;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    rc = check_hip(hipEventRecord(S->fork, stream), "fork record");
    bool used[kSideStreams] = {false, false, false};
    for (int i = 0; i < n && !rc; ++i) {
        hipStream_t s = stream;
        if (i > 0) {
            const int k = (i - 1) % kSideStreams;
            s = S->side[k];
            if (!used[k]) {
                rc = check_hip(hipStreamWaitEvent(s, S->fork, 0), "fork wait");
                used[k] = true;
            }
        }
        if (!rc) rc = launch(i, s);
    }
    // join every side stream that waited, also after a failed launch, so no
    // side stream is left inside a capture of `stream`
    for (int k = 0; k < kSideStreams; ++k) {
        if (!used[k]) continue;
        int r = check_hip(hipEventRecord(S->join[k], S->side[k]), "join record");
        if (!r) r = check_hip(hipStreamWaitEvent(stream, S->join[k], 0), "join wait");
        if (!rc) rc = r;
    }
    return rc;
}

// Annealing of every non-empty group.  Packed-row groups share one persistent
// launch; byte-state groups are launched per lanes-per-chain value.  The
// replay re-runs one chain per syndrome with the byte-state kernel, spreading
// a chain over more lanes when that is needed to give every CU several
// wavefronts.  Each launch has its own queue counter: d_counters[0] packed
// rows, [1..7] byte states by lanes per chain, [16..30] the kernels
// specialised to d = 3, 5, ..., 31, [40] random-site chains, [41..47] the
// planar kernels specialised to d = 3, 5, ..., 15, [48] ladders on the generic
// kernel, [49..55] and [31..38] ladders on the rotated kernels specialised to
// d = 3, ..., 15 and d = 17, ..., 31, [56..62] on the planar ones
// (d = 3, ..., 15); a replay (with its own d_counters base) uses [0] and [2].
static int launch_anneal(const xzzx_group *groups, const GroupWs *ws, int n_groups, AnnealMode mode,
                         uint64_t seed, int64_t unit_offset, int64_t units_override, uint32_t *d_counters,
                         hipStream_t stream, bool serial = false)
{
    std::vector<int> rows_sel;
    std::vector<int> bytes_sel[7];
    std::vector<int> static_sel[kStaticMaxD + 1];
    std::vector<int> replay_cp;   // replays starting from checkpoints: one chain per wavefront
    std::vector<int> site_sel;    // random-site plans: one chain (replay: syndrome) per lane
    std::vector<int> planar_sel[kPlanarStaticMaxD + 1];   // planar kernels specialised to d
    std::vector<int> gather_sel;  // replay: recoveries gathered from the states kept at E_min
    std::vector<int> ladder_sel;  // replica exchange: one chain per lane
    std::vector<int> ladder_rows_sel[kLadderRowsMaxD + 1];      // ... on the rotated kernels specialised to d
    std::vector<int> ladder_planar_sel[kPlanarStaticMaxD + 1];  // ... on the planar kernels specialised to d
    int64_t total_syn = 0;
    for (int i = 0; i < n_groups; ++i) {
        if (groups[i].n_syn <= 0) continue;
        const Plan &P = groups[i].plan->P;
        if (P.order == XZZX_ORDER_RANDOM_SITE || P.ladder_k ||
            (mode == AnnealMode::Replay && min_snap_words(groups[i]))) {
            if (mode == AnnealMode::Replay) gather_sel.push_back(i);
            else if (ladder_rows_d(groups[i])) ladder_rows_sel[ladder_rows_d(groups[i])].push_back(i);
            else if (ladder_planar_d(groups[i])) ladder_planar_sel[ladder_planar_d(groups[i])].push_back(i);
            else (P.ladder_k ? ladder_sel : site_sel).push_back(i);
            continue;
        }
        total_syn += groups[i].n_syn;
        if (mode != AnnealMode::Replay && P.use_rows && P.planar_d) planar_sel[P.planar_d].push_back(i);
        else if (mode != AnnealMode::Replay && uses_static(groups[i], unit_offset)) static_sel[P.static_d].push_back(i);
        else if (mode == AnnealMode::Replay && checkpoints_of(groups[i]) > 0) replay_cp.push_back(i);
        else if (mode != AnnealMode::Replay && P.use_rows && P.row_words) rows_sel.push_back(i);
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
        // groups that kept each chain's state at its E_min: gather
        for (int i : gather_sel) {
            if (rc) break;
            const xzzx_group &g = groups[i];
            const Plan &P = g.plan->P;
            const int64_t n = g.n_syn * (int64_t)P.lat.nq, nc = g.n_syn * 4 * (int64_t)g.n_rep;
            if ((n + 255) / 256 * 256 > kMaxLaunchItems) { set_error("too many recovery bytes in one group"); return XZZX_ERANGE; }
            const dim3 grid((unsigned)((n + 255) / 256));
            if (const int ld = ladder_rows_d(g))
                hipLaunchKernelGGL(k_static_recovery, grid, dim3(256), 0, stream, ws[i].min_snap,
                                   (int)min_snap_words(g), ws[i].best_chain, g.n_rep, ld, g.n_syn,
                                   2 * (ld + 1) <= 32 ? 1 : 2, g.d_recovery);
            else if (P.order == XZZX_ORDER_RANDOM_SITE || (P.ladder_k && !ladder_planar_d(g)))
                hipLaunchKernelGGL(k_site_recovery, grid, dim3(256), 0, stream, ws[i].min_snap, nc, ws[i].best_chain,
                                   g.n_rep, P.lat.nq, g.n_syn, g.d_recovery);
            else
                hipLaunchKernelGGL(k_rows_recovery, grid, dim3(256), 0, stream, ws[i].min_snap, (int)min_snap_words(g),
                                   ws[i].best_chain, g.n_rep, P.lat.nq, g.n_syn, P.ddev, P.row_words, g.d_recovery);
            rc = check_hip(hipGetLastError(), "recovery gather launch");
        }
        return rc;
    }
    // the launches of one call (one per kernel family and distance) run
    // concurrently: each alone may not fill the device (a mixed-distance batch
    // with a few hundred syndromes per distance)
    struct Set {
        const std::vector<int> *sel;
        bool rows;
        int lanes;
        uint32_t *counter;
        int static_d;
        bool site;
        int planar_d;
        bool ladder;
    };
    std::vector<Set> sets;
    if (!rows_sel.empty()) sets.push_back({&rows_sel, true, 1, d_counters, 0, false, 0, false});
    if (!site_sel.empty()) sets.push_back({&site_sel, false, 1, d_counters + 40, 0, true, 0, false});
    if (!ladder_sel.empty()) sets.push_back({&ladder_sel, false, 1, d_counters + 48, 0, false, 0, true});
    for (int d = 3; d <= kPlanarStaticMaxD; d += 2)
        if (!planar_sel[d].empty())
            sets.push_back({&planar_sel[d], true, 1, d_counters + 41 + (d - 3) / 2, 0, false, d, false});
    for (int d = 3; d <= kLadderRowsMaxD; d += 2)
        if (!ladder_rows_sel[d].empty())
            sets.push_back({&ladder_rows_sel[d], true, 1, d_counters + (d <= 15 ? 49 + (d - 3) / 2 : 31 + (d - 17) / 2),
                            d, false, 0, true});
    for (int d = 3; d <= kPlanarStaticMaxD; d += 2)
        if (!ladder_planar_sel[d].empty())
            sets.push_back({&ladder_planar_sel[d], true, 1, d_counters + 56 + (d - 3) / 2, 0, false, d, true});
    for (int d = kStaticMinD; d <= kStaticMaxD; d += 2)
        if (!static_sel[d].empty())
            sets.push_back({&static_sel[d], true, 1, d_counters + 16 + (d - kStaticMinD) / 2, d, false, 0, false});
    for (int l = 0; l < 7; ++l)
        if (!bytes_sel[l].empty())
            sets.push_back({&bytes_sel[l], false, 1 << l, d_counters + 1 + l, 0, false, 0, false});
    if (sets.size() <= 1 || mode == AnnealMode::Plain) {
        int rc = XZZX_OK;
        for (const Set &S : sets)
            if (!rc)
                rc = launch_set(groups, ws, *S.sel, S.rows, S.lanes, mode, seed, unit_offset, units_override, S.counter,
                                stream, S.static_d, S.site, S.planar_d, S.ladder);
        return rc;
    }
    return fork_join(stream, (int)sets.size(), [&](int i, hipStream_t s) {
        const Set &S = sets[i];
        return launch_set(groups, ws, *S.sel, S.rows, S.lanes, mode, seed, unit_offset, units_override, S.counter, s,
                          S.static_d, S.site, S.planar_d, S.ladder);
    }, serial);
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
    if (g.n_syn * kWave > kMaxLaunchItems) { set_error("too many syndromes in one group for one launch"); return XZZX_ERANGE; }
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)g.n_syn), dim3(kWave), 0, stream, A);
    return check_hip(hipGetLastError(), "k_reduce launch");
}

// The reference stage of the anneal-only entry point: the class of every
// caller reference relative to replica 0 (Alg. 7, Eqs. (35)-(36)), and, for
// groups that pass their syndromes, the check that every reference has
// syndrome S.  The check reads a flag back, so it synchronizes `stream` and
// is refused while `stream` is being captured.
static int check_references(const xzzx_group *groups, const GroupWs *ws, int n_groups, uint32_t *d_flag,
                            hipStream_t stream)
{
    bool any_syn = false;
    for (int i = 0; i < n_groups; ++i) any_syn |= groups[i].n_syn > 0 && groups[i].d_syn;
    if (any_syn) {
        hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
        int rc = check_hip(hipStreamIsCapturing(stream, &st), "hipStreamIsCapturing");
        if (rc) return rc;
        if (st != hipStreamCaptureStatusNone) {
            set_error("checking references against d_syn synchronizes the stream: not allowed under capture");
            return XZZX_EINVAL;
        }
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, stream, d_flag, 1);
        rc = check_hip(hipGetLastError(), "flag clear launch");
        if (rc) return rc;
    }
    for (int i = 0; i < n_groups; ++i) {
        const xzzx_group &g = groups[i];
        if (g.n_syn <= 0) continue;
        const int64_t blocks = g.n_syn * g.n_rep;
        for (int64_t b0 = 0; b0 < blocks; b0 += kMaxLaunchWaves) {
            const int64_t nb = std::min<int64_t>(kMaxLaunchWaves, blocks - b0);
            hipLaunchKernelGGL(k_ref_check, dim3((unsigned)nb), dim3(kWave), 0, stream, g.plan->P.ddev, ws[i].refs,
                               g.d_syn, g.n_rep, b0, ws[i].qraw, d_flag);
            const int rc = check_hip(hipGetLastError(), "k_ref_check launch");
            if (rc) return rc;
        }
        const int rc = launch_qcls(ws[i].qraw, g.n_syn, g.n_rep, ws[i].qcls, stream);
        if (rc) return rc;
    }
    if (!any_syn) return XZZX_OK;
    uint32_t bad = 0;
    int rc = check_hip(hipMemcpyAsync(&bad, d_flag, sizeof(bad), hipMemcpyDeviceToHost, stream), "flag read");
    if (!rc) rc = check_hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (rc) return rc;
    if (bad) { set_error("a reference's syndrome differs from the group's syndrome S"); return XZZX_EINVAL; }
    return XZZX_OK;
}

// serial: every launch on `stream`, in order, with no side streams or events
static int run_decode(const xzzx_group *groups, int n_groups, uint64_t greedy_seed, uint64_t anneal_seed,
                      int greedy_mode, int flags, void *d_workspace, size_t workspace_bytes,
                      hipStream_t stream, bool decode, bool serial = false)
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
    // the groups' greedy launches run concurrently (one group's launch alone
    // leaves the device idle in its tail)
    std::vector<int> gsel;
    for (int i = 0; i < n_groups; ++i)
        if (decode && groups[i].n_syn > 0 && (stages & XZZX_FLAG_STAGE_GREEDY)) gsel.push_back(i);
    rc = fork_join(stream, (int)gsel.size(), [&](int k, hipStream_t s) {
        const int i = gsel[k];
        const xzzx_group &g = groups[i];
        int r = launch_greedy(g.plan->P, g.d_syn, g.d_uid, g.n_syn, g.n_rep, greedy_seed, greedy_mode, ws[i].refs,
                              ws[i].qraw, s);
        if (!r) r = launch_qcls(ws[i].qraw, g.n_syn, g.n_rep, ws[i].qcls, s);
        return r;
    }, serial);
    if (rc) return rc;
    if (!decode && (stages & XZZX_FLAG_STAGE_GREEDY)) {
        rc = check_references(groups, ws.data(), n_groups, counter + 63, stream);
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
        rc = launch_anneal(groups, ws.data(), n_groups, AnnealMode::Persistent, anneal_seed, 0, -1, counter, stream,
                           serial);
        if (rc) return rc;
    }
    if (!(stages & XZZX_FLAG_STAGE_FINISH)) return XZZX_OK;
    for (int i = 0; i < n_groups; ++i) {
        rc = launch_reduce(groups[i], ws[i], stream);
        if (rc) return rc;
    }
    return launch_anneal(groups, ws.data(), n_groups, AnnealMode::Replay, anneal_seed, 0, -1, counter + 8, stream,
                         serial);
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
    const int lds = greedy_lds(P, (int64_t)n * n_rep <= kGreedyCacheWaves, &A);
    hipLaunchKernelGGL(greedy_split(P) ? k_greedy<true> : k_greedy<false>, dim3((unsigned)(n * n_rep)), dim3(kWave),
                       lds, stream, A);
    return check_hip(hipGetLastError(), "serving greedy launch");
}

int serve_slice(const ServeLaunch *launches, int n_launches, uint64_t seed, hipStream_t stream)
{
    const uint32_t lo = (uint32_t)seed, hi = (uint32_t)(seed >> 32);
    // the launches' tasks are consecutive: stash the start states of them all
    int n_tasks = 0;
    for (int i = 0; i < n_launches; ++i) n_tasks += launches[i].n;
    if (n_tasks > 0) {
        hipLaunchKernelGGL(k_serve_stash, dim3((unsigned)n_tasks), dim3(256), 0, stream, launches[0].tasks);
        const int rc = check_hip(hipGetLastError(), "serving stash launch");
        if (rc) return rc;
    }
    auto one = [&](int i, hipStream_t s) -> int {
        const ServeLaunch &L = launches[i];
        if (L.n <= 0) return XZZX_OK;
        if (L.kind == 0) {
            hipLaunchKernelGGL(k_serve_rows, dim3((unsigned)L.n), dim3(kWave), L.lds, s, L.tasks, lo, hi);
        } else if (L.kind == 1) {
            hipLaunchKernelGGL(k_serve_bytes, dim3((unsigned)L.n), dim3(kWave), L.lds, s, L.tasks, lo, hi);
        } else {
            const ServeKernel k = static_serve_kernel(L.d);
            if (!k) { set_error("no specialised serving kernel for this distance"); return XZZX_EINVAL; }
            hipLaunchKernelGGL(k, dim3((unsigned)L.n), dim3(kWave), 0, s, L.tasks, lo, hi);
        }
        return check_hip(hipGetLastError(), "serving slice launch");
    };
    // the kernels of one slice (one per family and distance) run concurrently
    if (n_launches <= 1) return n_launches ? one(0, stream) : XZZX_OK;
    return fork_join(stream, n_launches, one);
}

int run_concurrently(hipStream_t stream, int n, const std::function<int(int, hipStream_t)> &launch)
{
    if (n <= 1) return n ? launch(0, stream) : XZZX_OK;
    return fork_join(stream, n, launch);
}

int serve_finish(const ServeFinish *d_fin, const ServeTask *d_replay, int n, size_t lds_replay, uint64_t seed,
                 hipStream_t stream)
{
    if (n <= 0) return XZZX_OK;
    hipLaunchKernelGGL(k_serve_reduce, dim3((unsigned)n), dim3(kWave), 0, stream, d_fin);
    hipLaunchKernelGGL(k_serve_replay, dim3((unsigned)n), dim3(kWave), lds_replay, stream, d_replay,
                       (uint32_t)seed, (uint32_t)(seed >> 32));
    hipLaunchKernelGGL(k_serve_gather, dim3((unsigned)n), dim3(kWave), 0, stream, d_fin);
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
    if (blocks * 256 > kMaxLaunchItems) { set_error("batch too large for one launch (2^32 work-items)"); return XZZX_ERANGE; }
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

// ---- decode without allocation ----
// The workspace of xzzx_decode_noalloc: one array per device, resident from
// the library's load on that device until the process ends.  Host code never
// passes the array's name to a kernel (in host code it is only a stand-in for
// the symbol): it uses the device address that hipGetSymbolAddress returns,
// looked up once per device.
static __device__ __align__(256) uint8_t scratch[XZZX_NOALLOC_SCRATCH_BYTES];

static int scratch_address(void **out)
{
    static std::mutex mu;
    static void *addr[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) { set_error("hipGetDevice failed"); return XZZX_EDEVICE; }
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        const int rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
        if (rc) return rc;
        if (!p) { set_error("hipGetSymbolAddress returned NULL"); return XZZX_EDEVICE; }
        addr[dev] = p;
    }
    *out = addr[dev];
    return XZZX_OK;
}

extern "C" {

int xzzx_decode_noalloc(const xzzx_group *groups, int n_groups, uint64_t greedy_seed, uint64_t anneal_seed,
                        int greedy_mode, int flags, void *stream)
{
    size_t need = 0;
    int rc = xzzx_decode_workspace(groups, n_groups, &need);
    if (rc) return rc;
    if (need > (size_t)XZZX_NOALLOC_SCRATCH_BYTES) {
        set_error("workspace of these groups exceeds XZZX_NOALLOC_SCRATCH_BYTES");
        return XZZX_ERANGE;
    }
    void *ws = nullptr;
    rc = scratch_address(&ws);
    if (rc) return rc;
    return run_decode(groups, n_groups, greedy_seed, anneal_seed, greedy_mode, flags, ws,
                      (size_t)XZZX_NOALLOC_SCRATCH_BYTES, (hipStream_t)stream, true, true);
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
    // the stream's side streams and events exist before the capture begins
    SideSet *side = nullptr;
    int rc = side_set(s, &side);
    if (rc) return rc;
    rc = check_hip(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
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
