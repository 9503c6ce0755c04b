// Device-side code shared by the translation units of the gfx950 kernels:
// Philox, the chain jobs, the annealing cores (byte-state, packed-row and the
// packed-row core specialised to a distance) and the kernel bodies built on
// them.  Only inline functions and templates live here; each kernel is
// instantiated in exactly one translation unit.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

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

// Sum over the G = 2^LOGG lanes of one chain (lanes c*G .. c*G+G-1 of the
// wavefront), left in every one of them.  Each step doubles the group over
// which every lane holds the sum: DPP quad permutations (pairs, quads), the
// half-row and row mirrors (8 and 16 lanes: the mirrored lane lies in the
// other half), then the row swaps across 16 and 32 lanes.  All VALU, no LDS
// round trip (a shuffle would go through ds_bpermute), which matters on the
// latency-bound serving path where a chain spans the whole wavefront.
template <int LOGG>
__device__ __forceinline__ int32_t chain_sum(int32_t v)
{
    if constexpr (LOGG >= 1) v += __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    if constexpr (LOGG >= 2) v += __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    if constexpr (LOGG >= 3) v += __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    if constexpr (LOGG >= 4) v += __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false);  // row_mirror
    if constexpr (LOGG >= 5) {
        const auto p = __builtin_amdgcn_permlane16_swap((uint32_t)v, (uint32_t)v, false, false);
        v = (int32_t)(p[0] + p[1]);
    }
    if constexpr (LOGG >= 6) {
        const auto p = __builtin_amdgcn_permlane32_swap((uint32_t)v, (uint32_t)v, false, false);
        v = (int32_t)(p[0] + p[1]);
    }
    return v;
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
    // checkpoints of the specialised packed-row kernel (word-major planes of
    // lattice rows 0..d-1, plane stride cp_stride chains)
    uint32_t *cp_out;      // anneal: checkpoint planes to write (nullable), base of checkpoint 0
    const uint32_t *cp_in; // replay: packed rows to start from instead of src (nullable)
    int64_t cp_stride;     // chains per word plane
    int32_t cp_words;      // words per row of the checkpoint planes
    int32_t t0;            // first sweep to run (replay from a checkpoint)
    // serving: states kept for the replay of the chain's E_min phase (see
    // kept_entry); all wave-uniform bases, so nothing per lane stays live
    // through a sweep loop for them; nullable
    int32_t *cp_meta;      // the chains' entries
    uint8_t *cp_base;      // byte states: buffer b of chain ci at cp_base + b cp_bstride + ci nq
    int64_t cp_bstride;
    uint32_t *cp_packed;   // packed rows: buffer b of chain ci at cp_packed + (b nc + ci) cp_pwords
    int64_t cp_nc;
    int32_t cp_pwords;
    int32_t cp_meta0;      // the chain's entry at the range start (-1: the references)
    bool raw;              // replay: src holds the chain's own state (logical already applied)
};

// Serving keeps, per chain, two buffers of byte states and two of packed
// rows (the specialised kernel's layout), and one entry naming the state a
// replay of the chain's E_min phase starts from: -1 for the references at
// sweep 0, else (sweep << 2) | (packed << 1) | b.  Kept states go to buffer
// kept_scratch(entry) -- the one the entry does not name -- of either kind:
// the start state of a sweep range (bytes, by k_serve_stash), and inside a
// range the state every kServeCheckpointEvery sweeps (bytes from the
// byte-state kernel, packed rows from the specialised one).  When E_min has
// improved since the last kept state, the entry is made to name it.
__device__ __forceinline__ int kept_scratch(int32_t entry) { return entry >= 0 ? 1 - (entry & 1) : 0; }
__device__ __forceinline__ int32_t kept_entry(int sweep, bool packed, int b)
{
    return sweep == 0 ? -1 : ((sweep << 2) | ((packed ? 1 : 0) << 1) | b);
}

// Commit of a packed-row core's last kept state (at sweep sub; packed rows
// unless it is the range start) if E_min improved after it (stop past sweep
// sub's first phase).  The entry is re-read here rather than kept live
// through the sweep loop (only this chain writes it); a range from sweep 0
// sets it to -1 first.  Returns the entry.  (Copying the range's start
// state inside these kernels, before the sweeps or after them, was measured
// to cost the sweep loop up to 18 registers and spills at d = 9-11, so
// k_serve_stash does it before a slice.)
__device__ __forceinline__ int32_t commit_kept_state(const ChainJob &J, int sub, bool packed, int32_t stop)
{
    int32_t *entry = J.cp_meta + J.ci;
    int32_t e = *entry;
    if (stop > 4 * sub) {
        e = kept_entry(sub, packed, kept_scratch(e));
        *entry = e;
    }
    return e;
}

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
    uint32_t *min_snap;           // each chain's state at its first E_min: random-site kernel, packed
                                  // words [word][n_chains]; planar kernel specialised to d, its rows
                                  // [n_chains][planar_state_words(d)]
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
    j.cp_words = G.plan->static_words;
    j.t0 = 0;
    j.cp_meta = nullptr;
    j.cp_base = nullptr;
    j.cp_bstride = 0;
    j.cp_packed = nullptr;
    j.cp_nc = 0;
    j.cp_pwords = 0;
    j.cp_meta0 = -1;
    j.raw = false;
    if (replay && G.cp_rows && j.target > 0) {
        // start from the last checkpoint at or before the sweep of the target phase
        const int t_target = (j.target - 1) >> 2;
        const int n_cp = t_target / G.cp_every;
        if (n_cp > 0) {
            j.cp_in = G.cp_rows + (int64_t)(n_cp - 1) * G.plan->d * G.plan->static_words * G.n_chains + ci;
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
__device__ inline void bytes_core(const PlanDev *pl, const ChainJob &J, int t_begin, int t_end, uint32_t seed_lo,
                           uint32_t seed_hi, uint8_t *smem)
{
    constexpr int LOGC = 6 - LOGG;
    const int lane = threadIdx.x;
    const int c = lane >> LOGG;          // chain slot in this wavefront
    const int gl = lane & ((1 << LOGG) - 1);
    const int nq = pl->nq, M = pl->M, nblk = pl->nblk, nranks = pl->nranks;
    const uint32_t kneg = (uint32_t)pl->kneg;
    // a chain with at least as many lanes as a class has moves runs one move
    // per lane, else whole Philox blocks per lane (same draws, same chain)
    const bool per_move = LOGG >= 2 && M <= (1 << LOGG);
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
            // checkpoint rows (rotated lattice): qubit x of row y at bits 2x, 2x + 1
            const int y = q / dd, x = q - y * dd;
            const int64_t plane = (int64_t)y * J.cp_words + (x >> 4);
            v = J.active ? (J.cp_in[plane * J.cp_stride] >> (2 * (x & 15))) & 3u : 0u;
        } else {
            v = J.active ? (J.src[q] & 3u) : 0u;
            if (!J.resume && !J.raw) {
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

    // the thresholds of sweep t + 1 are fetched from HBM while sweep t runs
    constexpr int kThrPerLane = (kMaxRanks + kWave - 1) / kWave;
    uint32_t thr_next[kThrPerLane];
    auto fetch_thr = [&](int t) {
#pragma unroll
        for (int j = 0; j < kThrPerLane; ++j) {
            const int i = lane + j * kWave;
            thr_next[j] = (t < t_end && i < nranks) ? pl->thr[(size_t)t * nranks + i] : 0u;
        }
    };
    fetch_thr(t_begin);

    // serving: the state at the start of every kServeCheckpointEvery sweeps
    // is kept in the chain's scratch buffer (sb); when E_min has improved
    // since that start, the entry is committed to it and the other buffer
    // becomes the scratch.  A sub-range starting at sweep 0 commits the
    // references (-1) and needs no stored state.
    const bool keep = !REPLAY && J.cp_meta != nullptr;
    int32_t meta = J.cp_meta0;
    int sb = kept_scratch(meta);
    int sub = t_begin;
    // one-move-per-lane form: the Philox block of the coming phase
    uint4 rnd_pm = make_uint4(0u, 0u, 0u, 0u);
    if (per_move)
        rnd_pm = philox4x32_10(make_uint4(uid, cc, 4u * (uint32_t)t_begin, (uint32_t)gl >> 2), seed_lo, seed_hi);

    for (int t = t_begin; t < t_end && 4 * t < last_phase; ++t) {
        if (keep && t > sub && (t - t_begin) % kServeCheckpointEvery == 0) {
            if (stop > 4 * sub) {
                meta = kept_entry(sub, false, sb);
                if (sub > 0) sb ^= 1;
            }
            if (J.active) save_state(J.cp_base + sb * J.cp_bstride + J.ci * nq);
            sub = t;
        }
#pragma unroll
        for (int j = 0; j < kThrPerLane; ++j)
            if (lane + j * kWave < nranks) et_s[lane + j * kWave].y = (int)thr_next[j];
        wave_lds_fence();
        fetch_thr(t + 1);
        for (int k = 0; k < 4; ++k) {
            const uint2 *dk = desc_s + k * M;
            int32_t acc_de = 0;
            if (per_move) {
                // one move per lane: lane gl takes move gl of the class, with
                // word gl mod 4 of the class's Philox block gl / 4 (the four
                // lanes of a block each draw it, side by side).  The moves of
                // a class touch disjoint qubits, so each lane's loads and
                // stores are independent of the others'; this halves the
                // sequential LDS work of a phase against whole blocks per lane.
                // The block of the next phase (counter 4t + k + 1) is drawn
                // here, so its multiplies overlap this phase's LDS round trips.
                const uint4 rnd = rnd_pm;
                rnd_pm = philox4x32_10(make_uint4(uid, cc, 4u * (uint32_t)t + (uint32_t)k + 1u, (uint32_t)gl >> 2),
                                       seed_lo, seed_hi);
                const uint32_t sw = (uint32_t)gl & 3u;
                const uint32_t u = sw == 0 ? rnd.x : sw == 1 ? rnd.y : sw == 2 ? rnd.z : rnd.w;
                const uint2 d = dk[min(gl, M - 1)];
                const uint32_t a0 = ((d.x & 0xFFFFu) << LOGC) + c, a1 = ((d.x >> 16) << LOGC) + c;
                const uint32_t a2 = ((d.y & 0xFFFFu) << LOGC) + c, a3 = (((d.y >> 16) & 0x7FFu) << LOGC) + c;
                const uint32_t c0 = st[a0], c1 = st[a1], c2 = st[a2], c3 = st[a3];
                const uint32_t pat = c0 | (c1 << 2) | (c2 << 4) | (c3 << 6);
                const uint32_t rank = lut_s[((d.y >> 27) << 8) | pat];
                const int2 et = et_s[rank];
                if (gl < M && (rank < kneg || u < (uint32_t)et.y)) {
                    st[a0] = (uint8_t)(c0 ^ 2u);
                    st[a1] = (uint8_t)(c1 ^ 1u);
                    st[a2] = (uint8_t)(c2 ^ 1u);
                    st[a3] = (uint8_t)(c3 ^ 2u);
                    acc_de = et.x;
                }
            } else
            for (int b = gl; b < nblk; b += (1 << LOGG)) {
                const uint4 rnd = philox4x32_10(make_uint4(uid, cc, 4u * (uint32_t)t + (uint32_t)k, (uint32_t)b),
                                                seed_lo, seed_hi);
                const uint32_t uw[4] = {rnd.x, rnd.y, rnd.z, rnd.w};
                // The four moves of a block act on disjoint qubits (one colour
                // class), so all their loads are issued before any store; the
                // block's tail beyond M repeats the class's last move, which is
                // never applied.
                uint2 dw[4];
                uint32_t pat[4], rank[4];
#pragma unroll
                for (int w = 0; w < 4; ++w) dw[w] = dk[min(4 * b + w, M - 1)];
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const uint2 d = dw[w];
                    const uint32_t c0 = st[((d.x & 0xFFFFu) << LOGC) + c];
                    const uint32_t c1 = st[((d.x >> 16) << LOGC) + c];
                    const uint32_t c2 = st[((d.y & 0xFFFFu) << LOGC) + c];
                    const uint32_t c3 = st[(((d.y >> 16) & 0x7FFu) << LOGC) + c];
                    pat[w] = c0 | (c1 << 2) | (c2 << 4) | (c3 << 6);
                }
#pragma unroll
                for (int w = 0; w < 4; ++w) rank[w] = lut_s[((dw[w].y >> 27) << 8) | pat[w]];
                int2 ets[4];
#pragma unroll
                for (int w = 0; w < 4; ++w) ets[w] = et_s[rank[w]];
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const int2 et = ets[w];
                    if (4 * b + w < M && (rank[w] < kneg || uw[w] < (uint32_t)et.y)) {
                        const uint2 d = dw[w];
                        st[((d.x & 0xFFFFu) << LOGC) + c] = (uint8_t)((pat[w] & 3u) ^ 2u);
                        st[((d.x >> 16) << LOGC) + c] = (uint8_t)(((pat[w] >> 2) & 3u) ^ 1u);
                        st[((d.y & 0xFFFFu) << LOGC) + c] = (uint8_t)(((pat[w] >> 4) & 3u) ^ 1u);
                        st[(((d.y >> 16) & 0x7FFu) << LOGC) + c] = (uint8_t)((pat[w] >> 6) ^ 2u);
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
            if (keep) {
                if (stop > 4 * sub) meta = kept_entry(sub, false, sb);
                J.cp_meta[J.ci] = meta;
            }
        }
        if (J.states) save_state(J.states + (size_t)J.ci * nq);
    }
    wave_lds_fence();
}

// ---------------------------------------------------------------------------
// Random-site core (Algs. 2-3 as printed): every step picks one generator
// uniformly at random, so the steps of a chain are sequential and the
// parallelism is across chains: one chain per lane, 64 per wavefront.  The
// state of chain c is packed 2 bits per qubit, qubit q at bits 2 (q mod 16)
// of word q div 16, and word w of chain c at LDS word 64 w + c: whatever
// qubits the lanes pick, one instruction's accesses fall in distinct banks.
// Position nq is scratch for absent generator slots.  Step m of sweep t uses
// Philox(uid, chain, 2^31 + t, m div 2): words 2 (m mod 2) and 2 (m mod 2) + 1
// are the site draw (site = floor(u N_stab / 2^32), face-id order) and the
// acceptance draw.  E_min is tracked after every step; stop = t N_stab + m + 1
// (0 = the start), and the state at the first E_min is kept in `snap` (word w
// of chain ci at snap[w * snap_stride + ci]) for the recovery.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int site_words(int nq) { return nq / 16 + 1; }

__device__ inline void site_core(const PlanDev *pl, const ChainJob &J, uint32_t seed_lo, uint32_t seed_hi,
                                 uint8_t *smem, uint32_t *snap, int64_t snap_stride)
{
    const int c = threadIdx.x;
    const int nq = pl->nq, nstab = pl->nstab, nranks = pl->nranks, n_sweeps = pl->n_sweeps;
    const uint32_t kneg = (uint32_t)pl->kneg;
    int32_t W[4];
    W[0] = pl->W[0]; W[1] = pl->W[1]; W[2] = pl->W[2]; W[3] = pl->W[3];
    const LdsLayout lo = lds_layout(pl->M, pl->ntypes, nranks);
    const uint2 *desc_s = reinterpret_cast<const uint2 *>(smem + lo.desc);   // by face id
    const uint8_t *lut_s = smem + lo.lut;
    int2 *et_s = reinterpret_cast<int2 *>(smem + lo.et);
    uint32_t *st = reinterpret_cast<uint32_t *>(smem + lo.state);
    const int nw = site_words(nq);
    const uint32_t uid = J.uid, cc = J.cc;

    const bool use_x = (J.lp == 1 || J.lp == 2), use_z = (J.lp == 2 || J.lp == 3);
    int32_t E = 0;
    for (int w = 0; w < nw; ++w) {
        uint32_t word = 0;
        for (int i = 0; i < 16; ++i) {
            const int q = 16 * w + i;
            if (q >= nq) break;
            uint32_t v = J.active ? (J.src[q] & 3u) : 0u;
            if (use_x) v ^= pl->lx[q];
            if (use_z) v ^= pl->lz[q];
            word |= v << (2 * i);
            E += weight_of(W, v);
        }
        st[w * kWave + c] = word;
    }
    int32_t Emin = E, stop = 0;
    wave_lds_fence();

    auto save_state = [&](uint8_t *dst) {
        for (int q = 0; q < nq; ++q) dst[q] = (uint8_t)((st[(q >> 4) * kWave + c] >> (2 * (q & 15))) & 3u);
    };
    auto keep_min = [&]() {
        for (int w = 0; w < nw; ++w) snap[(int64_t)w * snap_stride + J.ci] = st[w * kWave + c];
    };
    const bool keep = snap != nullptr && J.active;
    if (keep) keep_min();

    constexpr int kThrPerLane = (kMaxRanks + kWave - 1) / kWave;
    uint32_t thr_next[kThrPerLane];
    auto fetch_thr = [&](int t) {
#pragma unroll
        for (int j = 0; j < kThrPerLane; ++j) {
            const int i = c + j * kWave;
            thr_next[j] = (t < n_sweeps && i < nranks) ? pl->thr[(size_t)t * nranks + i] : 0u;
        }
    };
    fetch_thr(0);

    auto step = [&](uint32_t u_site, uint32_t u_acc, int32_t s) {
        const uint32_t f = __umulhi(u_site, (uint32_t)nstab);
        const uint2 d = desc_s[f];
        const uint32_t q0 = d.x & 0xFFFFu, q1 = d.x >> 16, q2 = d.y & 0xFFFFu, q3 = (d.y >> 16) & 0x7FFu;
        uint32_t *a0 = st + (q0 >> 4) * kWave + c, *a1 = st + (q1 >> 4) * kWave + c;
        uint32_t *a2 = st + (q2 >> 4) * kWave + c, *a3 = st + (q3 >> 4) * kWave + c;
        const uint32_t s0 = 2u * (q0 & 15u), s1 = 2u * (q1 & 15u), s2 = 2u * (q2 & 15u), s3 = 2u * (q3 & 15u);
        const uint32_t pat = ((*a0 >> s0) & 3u) | (((*a1 >> s1) & 3u) << 2) | (((*a2 >> s2) & 3u) << 4) |
                             (((*a3 >> s3) & 3u) << 6);
        const uint32_t rank = lut_s[((d.y >> 27) << 8) | pat];
        const int2 et = et_s[rank];
        if (rank < kneg || u_acc < (uint32_t)et.y) {
            // slots 0 and 3 carry X, slots 1 and 2 carry Z; slots of one
            // generator may share a word, so each is read, flipped and written
            *a0 ^= 2u << s0;
            *a1 ^= 1u << s1;
            *a2 ^= 1u << s2;
            *a3 ^= 2u << s3;
            E += et.x;
        }
        if (E < Emin) {
            Emin = E;
            stop = s + 1;
            if (keep) keep_min();
        }
    };

    for (int t = 0; t < n_sweeps; ++t) {
#pragma unroll
        for (int j = 0; j < kThrPerLane; ++j)
            if (c + j * kWave < nranks) et_s[c + j * kWave].y = (int)thr_next[j];
        wave_lds_fence();
        fetch_thr(t + 1);
        const int32_t s0 = t * nstab;
        for (int m = 0; m < nstab; m += 2) {
            const uint4 r = philox4x32_10(make_uint4(uid, cc, 0x80000000u + (uint32_t)t, (uint32_t)m >> 1),
                                          seed_lo, seed_hi);
            step(r.x, r.y, s0 + m);
            if (m + 1 < nstab) step(r.z, r.w, s0 + m + 1);
        }
        wave_lds_fence();
    }
    if (J.active) {
        J.emin[J.ci] = Emin;
        J.stop[J.ci] = stop;
        J.efin[J.ci] = E;
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
__device__ inline void rows_core(const PlanDev *pl, const ChainJob &J, int t_begin, int t_end, uint32_t seed_lo,
                          uint32_t seed_hi, uint8_t *smem)
{
    const int lane = threadIdx.x;
    const int nq = (int)uni(pl->nq), nblk = (int)uni(pl->nblk);
    const int nranks = (int)uni(pl->nranks), ntypes = (int)uni(pl->ntypes);
    const uint32_t kneg = uni(pl->kneg);
    const int rows = (int)uni(pl->rows);
    const int Mpad = 4 * nblk;
    int32_t W[4];
    W[0] = 0; W[1] = (int32_t)uni(pl->W[1]); W[2] = (int32_t)uni(pl->W[2]); W[3] = (int32_t)uni(pl->W[3]);
    const RowsLds lo = rows_layout(ntypes, nranks);
    const uint8_t *lut_s = smem + lo.lut;
    int2 *et_s = reinterpret_cast<int2 *>(__builtin_assume_aligned(smem + lo.et, 8));
    uint32_t *rw = reinterpret_cast<uint32_t *>(smem + lo.rows) + lane;   // this lane's column
    const uint32_t uid = J.uid, cc = J.cc;
    const bool use_x = !J.resume && (J.lp == 1 || J.lp == 2), use_z = !J.resume && (J.lp == 2 || J.lp == 3);

    // serving: a fresh request's replay entries start at the references
    if (J.cp_meta && t_begin == 0 && J.active) J.cp_meta[J.ci] = -1;
    // pack the state into rows (qubit q at row qpos >> 8, column qpos & 0xFF);
    // E of the state on the way
    int32_t E = 0;
    for (int i = 0; i < rows * NW; ++i) rw[i * kWave] = 0;
    for (int q = 0; q < nq; ++q) {
        const uint32_t p = uni(pl->qpos[q]);
        uint32_t v = J.active ? (J.src[q] & 3u) : 0u;
        if (use_x) v ^= pl->lx[q];
        if (use_z) v ^= pl->lz[q];
        if (!J.active) v = 0u;
        rw[((p >> 8) * NW + ((p & 0xFFu) >> 4)) * kWave] |= v << (2 * (p & 15u));
        E += weight_of(W, v);
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
        if (J.cp_meta) commit_kept_state(J, t_begin, false, stop);
        if (J.states) {
            uint8_t *dst = J.states + (size_t)J.ci * nq;
            for (int q = 0; q < nq; ++q) {
                const uint32_t p = uni(pl->qpos[q]);
                const uint32_t word = rw[((p >> 8) * NW + ((p & 0xFFu) >> 4)) * kWave];
                dst[q] = (uint8_t)((word >> (2 * (p & 15u))) & 3u);
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
__device__ inline void load_static_tables(const PlanDev *pl, uint16_t *lut_s, uint4 *et_s)
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

// Acceptance mask of a move of the specialised kernels: all ones iff
// u < thr or the move always accepts (dE <= 0: always = all ones, and its
// table threshold is 0, so the borrow of u - thr is 0).  Two instructions:
// the borrow of u - thr goes through the carry into always - 0 - borrow.
__device__ __forceinline__ uint32_t accept_sel(uint32_t u, uint32_t thr, uint32_t always)
{
    unsigned int borrow, unused;
    (void)__builtin_subc(u, thr, 0u, &borrow);
    return __builtin_subc(always, 0u, borrow, &unused);
}

// Rows of the specialised kernel: the d lattice rows only, qubit x of a row
// at bits 2x, 2x + 1, and one spare column (x = d) at the right end that the
// right-boundary generators may flip (its bits are never read as a qubit).
// 2(d + 1) bits: one word for d <= 15, two for d <= 31.
template <int D>
struct StaticRows {
    static constexpr int NW = 2 * (D + 1) <= 32 ? 1 : 2;
    static constexpr int N = D * NW;   // registers per chain; word w of lattice row y at [y * NW + w]
};

// Bits [BO - S, BO - S + 31] of row word pair (hi:lo) of a row, for a shift
// S in [0, 5]: the nibble at BO lands at bit S.  BO = -2 is the nibble of
// the left-boundary generators, whose missing column reads as zero.  A
// nibble may straddle the two words of a row (BO = 30).
template <int NW, int BO, int S>
__device__ __forceinline__ uint32_t row_bits(const uint32_t *w)
{
    if constexpr (NW == 1 || BO + 3 < 32) {
        return BO >= S ? w[0] >> (BO - S) : w[0] << (S - BO);
    } else if constexpr (BO >= 32) {
        return BO - 32 >= S ? w[1] >> (BO - 32 - S) : (w[1] << (S - (BO - 32))) | (w[0] >> (32 - (S - (BO - 32))));
    } else {
        return __builtin_amdgcn_alignbit(w[1], w[0], BO - S);
    }
}

// A 32-bit constant materialised in a scalar register where it is used.
// Large lattices use dozens of distinct flip masks; left to itself the
// compiler hoists them all out of the sweep loop and spills the surplus.
template <uint32_t C>
__device__ __forceinline__ uint32_t sreg_const()
{
    uint32_t v;
    asm volatile("s_mov_b32 %0, %1" : "=s"(v) : "i"(C));
    return v;
}

// w ^= (MASK << BO) & sel over the words of one row (MASK: 4 bits; for
// BO = -2 the bits of the missing column drop out)
template <int NW, int BO, uint32_t MASK>
__device__ __forceinline__ void row_flip_static(uint32_t *w, uint32_t sel)
{
    constexpr uint64_t m = BO >= 0 ? (uint64_t)MASK << BO : (uint64_t)(MASK >> -BO);
    if constexpr (NW == 1) {
        w[0] = xor_and(w[0], (uint32_t)m, sel);
    } else {
        if constexpr ((uint32_t)m != 0u) w[0] = xor_and(w[0], sreg_const<(uint32_t)m>(), sel);
        if constexpr ((uint32_t)(m >> 32) != 0u) w[1] = xor_and(w[1], sreg_const<(uint32_t)(m >> 32)>(), sel);
    }
}

// Generator W of Philox block B of colour class K: cell (i, j) covers
// lattice rows j (slots 0, 1) and j + 1 (slots 2, 3), nibble of columns
// i, i + 1 at bit 2i; rows -1 and d do not exist.
template <int D, int K, int B, int W>
struct StaticGen {
    static constexpr RotGen g = RotSchedule<D>{}.g[K][4 * B + W];
    static constexpr bool real = g.shp != 5;
    static constexpr int ya = g.Y - 1, BO = g.bo - 2;
    static constexpr bool has_a = ya >= 0, has_b = ya + 1 < D;
};

// The move's energy-table entry, looked up from its 8-bit slot pattern.
template <int D, int K, int B, int W>
__device__ __forceinline__ uint4 static_lookup(const uint32_t (&r)[StaticRows<D>::N], const uint16_t *lut_s,
                                               const uint4 *et_s)
{
    using G = StaticGen<D, K, B, W>;
    constexpr int NW = StaticRows<D>::NW;
    if constexpr (!G::real) {
        return make_uint4(0u, 0u, 0u, 0u);
    } else {
        const uint32_t *ra = r + (G::has_a ? G::ya : 0) * NW, *rb = r + (G::has_b ? G::ya + 1 : 0) * NW;
        uint32_t pat2 = 0;
        if constexpr (G::has_a) pat2 |= row_bits<NW, G::BO, 1>(ra) & 0x1Eu;
        if constexpr (G::has_b) pat2 |= row_bits<NW, G::BO, 5>(rb) & 0x1E0u;
        const uint32_t off = *reinterpret_cast<const uint16_t *>(reinterpret_cast<const uint8_t *>(lut_s) +
                                                                 512u * G::g.shp + pat2);
        return *reinterpret_cast<const uint4 *>(reinterpret_cast<const uint8_t *>(et_s) + off);
    }
}

// Acceptance of the move with draw u and entry e, its flips and energy.
template <int D, int K, int B, int W>
__device__ __forceinline__ void static_apply(uint32_t (&r)[StaticRows<D>::N], uint32_t u, const uint4 &e, int32_t &acc)
{
    using G = StaticGen<D, K, B, W>;
    constexpr int NW = StaticRows<D>::NW;
    if constexpr (G::real) {
        uint32_t *ra = r + (G::has_a ? G::ya : 0) * NW, *rb = r + (G::has_b ? G::ya + 1 : 0) * NW;
        // all ones on accepting lanes: u < threshold, or dE <= 0 (mask all
        // ones).  Up to d = 15 (eight wavefronts per SIMD) two instructions
        // through the carry, the table giving those ranks threshold 0; the
        // larger lattices, at four or five wavefronts, keep the
        // sign-extension form: the carry form's compare and borrow share one
        // condition register, which serialises the moves of a block, and
        // d = 31 ran 21 % slower with it
        uint32_t sel;
        if constexpr (D <= 15) sel = accept_sel(u, e.y, e.z);
        else sel = lt_mask(u, e.y) | e.z;
        if constexpr (G::has_a) row_flip_static<NW, G::BO, 6u>(ra, sel);   // X_left | Z_up
        if constexpr (G::has_b) row_flip_static<NW, G::BO, 9u>(rb, sel);   // Z_down | X_right
        acc += (int32_t)(e.x & sel);
    }
}

template <int D, int K, int B>
__device__ __forceinline__ void static_block(uint32_t (&r)[StaticRows<D>::N], const PhiloxHead &h, uint32_t k0, uint32_t k1,
                                             const uint16_t *lut_s, const uint4 *et_s, int32_t &acc)
{
    const uint4 u = philox_block(h, (uint32_t)B, k0, k1);
    // The four generators of a block belong to one colour class and act on
    // disjoint qubits: a flip of one leaves the others' slot bits as they
    // were, so all four look up their entries from the rows before any flip
    // and their LDS reads overlap (looked up one after another, each move's
    // pattern waited for the previous move's flips of the same row words).
    // Moves looked up together per group (measured per distance): four, but
    // one at a time at d = 15, where four entries in flight spill (and pairs
    // measured slower).
    constexpr int OV = D == 15 ? 1 : 4;
    if constexpr (OV == 1) {
        static_apply<D, K, B, 0>(r, u.x, static_lookup<D, K, B, 0>(r, lut_s, et_s), acc);
        static_apply<D, K, B, 1>(r, u.y, static_lookup<D, K, B, 1>(r, lut_s, et_s), acc);
        static_apply<D, K, B, 2>(r, u.z, static_lookup<D, K, B, 2>(r, lut_s, et_s), acc);
        static_apply<D, K, B, 3>(r, u.w, static_lookup<D, K, B, 3>(r, lut_s, et_s), acc);
    } else if constexpr (OV == 2) {
        const uint4 e0 = static_lookup<D, K, B, 0>(r, lut_s, et_s);
        const uint4 e1 = static_lookup<D, K, B, 1>(r, lut_s, et_s);
        static_apply<D, K, B, 0>(r, u.x, e0, acc);
        static_apply<D, K, B, 1>(r, u.y, e1, acc);
        const uint4 e2 = static_lookup<D, K, B, 2>(r, lut_s, et_s);
        const uint4 e3 = static_lookup<D, K, B, 3>(r, lut_s, et_s);
        static_apply<D, K, B, 2>(r, u.z, e2, acc);
        static_apply<D, K, B, 3>(r, u.w, e3, acc);
    } else {
        const uint4 e0 = static_lookup<D, K, B, 0>(r, lut_s, et_s);
        const uint4 e1 = static_lookup<D, K, B, 1>(r, lut_s, et_s);
        const uint4 e2 = static_lookup<D, K, B, 2>(r, lut_s, et_s);
        const uint4 e3 = static_lookup<D, K, B, 3>(r, lut_s, et_s);
        static_apply<D, K, B, 0>(r, u.x, e0, acc);
        static_apply<D, K, B, 1>(r, u.y, e1, acc);
        static_apply<D, K, B, 2>(r, u.z, e2, acc);
        static_apply<D, K, B, 3>(r, u.w, e3, acc);
    }
    // the energy change is summed block by block: left free, the compiler
    // reassociates the whole class's sum into a tree at the end of the class
    // and keeps every move's term live in a register until then.  The asm is
    // not volatile, so it orders only the sum: a volatile one also kept the
    // scheduler from moving the next block's work past it (d = 11 ran 3.5 %
    // slower)
    asm("" : "+v"(acc));
}

template <int D, int K, int... Bs>
__device__ __forceinline__ void static_class(uint32_t (&r)[StaticRows<D>::N], const PhiloxHead &h, uint32_t k0, uint32_t k1,
                                             const uint16_t *lut_s, const uint4 *et_s, int32_t &acc,
                                             std::integer_sequence<int, Bs...>)
{
    (static_block<D, K, Bs>(r, h, k0, k1, lut_s, et_s, acc), ...);
}

// One byte per qubit, row-major, from the specialised kernel's rows.
template <int D>
__device__ __forceinline__ void static_unpack(const uint32_t (&r)[StaticRows<D>::N], uint8_t *dst)
{
    constexpr int NW = StaticRows<D>::NW;
#pragma unroll
    for (int y = 0; y < D; ++y)
#pragma unroll
        for (int w = 0; w < NW; ++w)
#pragma unroll 1
            for (int x = 16 * w; x < min(D, 16 * w + 16); ++x)
                dst[y * D + x] = (uint8_t)((r[y * NW + w] >> (2 * (x - 16 * w))) & 3u);
}

// The chain's starting state packed into the specialised kernel's rows (the
// logical operators of its coset applied as asked), and its energy.
template <int D>
__device__ __forceinline__ int32_t static_load(const PlanDev *pl, const ChainJob &J, bool use_x, bool use_z,
                                               const int32_t (&W)[4], uint32_t (&r)[StaticRows<D>::N])
{
    constexpr int NW = StaticRows<D>::NW;
    int32_t E = 0;
#pragma unroll
    for (int y = 0; y < D; ++y) {
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            uint32_t word = 0;
            if (J.active) {
                // qubits x = 16 w .. 16 w + 15 of lattice row y; not unrolled:
                // a fully unrolled row would keep every byte load in flight
#pragma unroll 1
                for (int x = 16 * w; x < min(D, 16 * w + 16); ++x) {
                    const int q = y * D + x;
                    uint32_t v = J.src[q] & 3u;
                    if (use_x) v ^= pl->lx[q];
                    if (use_z) v ^= pl->lz[q];
                    word |= v << (2 * (x - 16 * w));
                    E += weight_of(W, v);
                }
            }
            r[y * NW + w] = word;
        }
    }
    return E;
}

template <int D>
__device__ __forceinline__ void rows_static_core(const PlanDev *pl, const ChainJob &J, int t_begin, int t_end, uint32_t seed_lo,
                                 uint32_t seed_hi, const uint16_t *lut_s, uint4 *et_s, int cp_interval)
{
    constexpr int NW = StaticRows<D>::NW;
    constexpr int NB = RotSchedule<D>::MP / 4;
    using Blocks = std::make_integer_sequence<int, NB>;
    const int lane = threadIdx.x;
    const int nranks = (int)uni(pl->nranks), kneg = (int)uni(pl->kneg);
    int32_t W[4];
    W[0] = 0; W[1] = (int32_t)uni(pl->W[1]); W[2] = (int32_t)uni(pl->W[2]); W[3] = (int32_t)uni(pl->W[3]);
    // a task's 64 chains belong to one syndrome
    const uint32_t uid = uni(J.uid), cc = J.cc;
    const uint32_t k0 = uni(seed_lo), k1 = uni(seed_hi);
    const bool use_x = !J.resume && (J.lp == 1 || J.lp == 2), use_z = !J.resume && (J.lp == 2 || J.lp == 3);
    // lane 0 is always active and a task's chains are consecutive: chain of lane l = ci0 + l
    const int64_t ci0 = (int64_t)(((uint64_t)uni((uint32_t)((uint64_t)J.ci >> 32)) << 32) | uni((uint32_t)J.ci));
    const int cp_every = J.cp_out ? cp_interval : 0;

    uint32_t r[StaticRows<D>::N];
    int32_t E = static_load<D>(pl, J, use_x, use_z, W, r);
    int32_t Emin = E, stop = 0;
    if (J.resume && J.active) {
        E = J.efin[J.ci];
        Emin = J.emin[J.ci];
        stop = J.stop[J.ci];
    }

    // serving: the state is also kept every kServeCheckpointEvery sweeps of
    // the range, for the replay (sub: sweep of the state kept last)
    const bool keep = J.cp_meta != nullptr;
    if (keep && t_begin == 0 && J.active) J.cp_meta[J.ci] = -1;
    int sub = t_begin;
    for (int t = t_begin; t < t_end;) {
        // sweeps up to the next checkpoint, then the checkpoint (the state at
        // the start of sweep t, every cp_every sweeps)
        int t_stop = t_end;
        if (cp_every) t_stop = min(t_end, (t / cp_every + 1) * cp_every);
        if (keep) t_stop = min(t_end, t_begin + ((t - t_begin) / kServeCheckpointEvery + 1) * kServeCheckpointEvery);
        for (; t < t_stop; ++t) {
            wave_lds_fence();
            // this sweep's thresholds (0 for the ranks with dE <= 0 where the
            // acceptance goes through the carry: see static_apply)
            if constexpr (D <= 15) {
                for (int i = lane; i < nranks; i += kWave) et_s[i].y = i < kneg ? 0u : pl->thr[(size_t)t * nranks + i];
            } else {
                for (int i = lane; i < nranks; i += kWave) et_s[i].y = pl->thr[(size_t)t * nranks + i];
            }
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
            uint32_t *cp = J.cp_out + (int64_t)(t / cp_every - 1) * (D * NW) * J.cp_stride + ci0 + lane;
#pragma unroll
            for (int i = 0; i < D * NW; ++i) cp[i * J.cp_stride] = r[i];
        }
        if (keep && t < t_end) {
            if (J.active) {
                const int32_t e = commit_kept_state(J, sub, sub != t_begin, stop);
                uint32_t *dst = J.cp_packed + (kept_scratch(e) * J.cp_nc + J.ci) * J.cp_pwords;
#pragma unroll
                for (int i = 0; i < D * NW; ++i) dst[i] = r[i];
            }
            sub = t;
        }
    }
    if (J.active) {
        J.emin[J.ci] = Emin;
        J.stop[J.ci] = stop;
        J.efin[J.ci] = E;
        if (keep) commit_kept_state(J, sub, sub != t_begin, stop);
        if (J.states) static_unpack<D>(r, J.states + (size_t)J.ci * (D * D));
    }
}

// ---------------------------------------------------------------------------
// Replica exchange (ladders of K fixed inverse temperatures; the paper names
// replica exchange as future work, Sec. VII).  Shared by the generic ladder
// kernel and the ladder kernels specialised to d.
// ---------------------------------------------------------------------------
// The exchange rule's threshold T(n) = floor(prod over the set bits i of n
// of R_i / 2^32), the product in 64-bit fixed point from 2^64 - 1.
__device__ __forceinline__ uint32_t swap_threshold(const uint64_t *R, uint32_t n)
{
    uint64_t p = ~0ull;
    // bits in ascending order, up to the highest set one
    int i = 0;
    for (uint32_t m = n; m != 0u; m >>= 1, ++i)
        if (m & 1u) p = __umul64hi(p, R[i]);
    return (uint32_t)(p >> 32);
}

// Tables of the ladder kernels specialised to d: the (shape, pattern) ->
// entry offset table of the annealing kernels, and one 16-byte entry
// (dE, threshold, always-accept mask) per (level, rank), the levels' tables
// one after another; ranks with dE <= 0 take threshold 0 (see accept_sel).
__device__ inline void load_ladder_tables(const PlanDev *pl, uint16_t *lut_s, uint4 *et_s)
{
    const int lane = threadIdx.x;
    const int nranks = pl->nranks, kneg = pl->kneg, K = pl->ladder_k;
    for (int i = lane; i < 256 * 6; i += kWave) lut_s[i] = (uint16_t)(16u * pl->lut[i]);
    for (int i = lane; i < K * nranks; i += kWave) {
        const int rk = i % nranks;
        const int32_t de = pl->dE[rk];
        et_s[i] = make_uint4((uint32_t)de, rk < kneg ? 0u : pl->ladder_thr[i], de <= 0 ? 0xFFFFFFFFu : 0u, 0u);
    }
    wave_lds_fence();
}

// Exchanges of adjacent levels after sweep t: pairs (k, k + 1) for k = t mod
// 2, t mod 2 + 2, ...; the pair's uniform is word p mod 4 of the Philox block
// (uid, 2^31 | ladder, t, p / 4), p = (k - t mod 2) / 2, and the pair swaps
// when the higher level's energy is not below the lower one's or when the
// uniform falls below T(E_low - E_high).  A lane's chain keeps its state and
// takes its partner's level.  The chains of one ladder and coset P hold the
// slots base + 4 level + P of the ladder's block of 4K lanes, a permutation
// of the block, so one forward permute tells every slot the lane holding it.
__device__ __forceinline__ int ladder_exchange(int level, int32_t E, int K, uint32_t P, uint32_t uid,
                                               uint32_t ladder_id, int t, uint32_t k0, uint32_t k1, const uint64_t *R)
{
    const int lane = threadIdx.x;
    const int base = lane & ~(4 * K - 1);
    const int holder = __builtin_amdgcn_ds_permute((base + 4 * level + (int)P) << 2, lane);
    const int par = t & 1;
    const bool low = ((level - par) & 1) == 0;
    const int plevel = low ? level + 1 : level - 1;
    const bool paired = plevel >= 0 && plevel < K;
    const int partner = __builtin_amdgcn_ds_bpermute((base + 4 * (paired ? plevel : level) + (int)P) << 2, holder);
    const int32_t ep = __builtin_amdgcn_ds_bpermute(partner << 2, E);
    if (paired) {
        const int32_t e_lo = low ? E : ep, e_hi = low ? ep : E;
        const uint32_t p = (uint32_t)((low ? level : plevel) - par) >> 1;
        const uint4 rr = philox4x32_10(make_uint4(uid, 0x80000000u | ladder_id, (uint32_t)t, p >> 2), k0, k1);
        const uint32_t u = (p & 3u) == 0 ? rr.x : (p & 3u) == 1 ? rr.y : (p & 3u) == 2 ? rr.z : rr.w;
        if (e_hi >= e_lo || u < swap_threshold(R, (uint32_t)(e_lo - e_hi))) return plevel;
    }
    return level;
}

// Task loop of the ladder kernels specialised to d (MODE 0: persistent
// wavefronts on the atomic task queue; 2: one task per workgroup), tasks of
// 64 consecutive chains.  The offset table is static LDS, so its address
// folds into each lookup's instruction; the K level tables are dynamic LDS
// (16 K n_ranks bytes).  core(G, J, lut_s, et_s) runs one lane's chain.
template <int MODE, typename Core>
__device__ __forceinline__ void ladder_static_body(const AnnealArgs &A, Core core)
{
    __shared__ uint16_t lut_s[256 * 6];
    extern __shared__ __align__(16) uint4 et_s[];
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
            load_ladder_tables(G.plan, lut_s, et_s);
            loaded = G.plan;
        }
        const ChainJob J = batch_job(G, unit0 + threadIdx.x, false);
        core(G, J, lut_s, et_s);
    }
}

__device__ inline void load_rows_tables(const PlanDev *pl, uint8_t *smem)
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

// by_face: descriptors in face-id order (random-site core) instead of by
// (colour class, rank)
__device__ inline void load_plan_tables(const PlanDev *pl, uint8_t *smem, bool by_face = false)
{
    const int lane = threadIdx.x;
    const LdsLayout lo = lds_layout(pl->M, pl->ntypes, pl->nranks);
    uint2 *desc_s = reinterpret_cast<uint2 *>(smem + lo.desc);
    const uint2 *desc_g = reinterpret_cast<const uint2 *>(by_face ? pl->face_desc : pl->desc);
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

// Batch body of the random-site core (MODE as in batch_kernel_body): tasks of
// 64 chains; the face descriptors are staged by face id.
template <int MODE>
__device__ __forceinline__ void site_kernel_body(const AnnealArgs &A)
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
        const int64_t unit0 = ((int64_t)task - G.task_begin) << 6;
        if (G.plan != loaded) {
            wave_lds_fence();
            load_plan_tables(G.plan, smem, true);
            loaded = G.plan;
        }
        const ChainJob J = batch_job(G, unit0 + threadIdx.x, false);
        site_core(G.plan, J, A.seed_lo, A.seed_hi, smem, G.min_snap, G.n_chains);
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

// Occupancy target of the specialised kernels (VGPR budget 512 / waves):
// eight wavefronts per SIMD hides the LDS and multiply latencies best
// (measured at d = 11: eight waves with a few spills beat seven without);
// with two words per row (d >= 17) the state alone takes 2d registers, so
// larger lattices run fewer wavefronts.
constexpr int static_waves(int d) { return d <= 15 ? 8 : d <= 21 ? 5 : 4; }

template <int D>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(static_waves(D), static_waves(D))))
void k_anneal_rows_d(AnnealArgs A) { static_rows_body<0, D>(A); }
template <int D>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(static_waves(D), static_waves(D))))
void k_anneal_rows_d_plain(AnnealArgs A) { static_rows_body<2, D>(A); }

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
    j.cp_words = 0;
    j.t0 = 0;
    // start states kept at sweep-range boundaries: buffer b of chain c at
    // cp + (b nc + c) nq; cpm[c] = (sweep << 1) | b of the one a replay of
    // the chain's E_min phase starts from, -1 for the references at sweep 0
    j.cp_meta = nullptr;
    j.cp_base = nullptr;
    j.cp_bstride = 0;
    j.cp_packed = nullptr;
    j.cp_nc = 0;
    j.cp_pwords = 0;
    j.cp_meta0 = -1;
    j.raw = false;
    if (T.cpm) {
        if (replay) {
            const int32_t meta = T.cpm[c];
            if (meta >= 0) {
                const int b = meta & 1;
                if (meta & 2) {   // packed rows of the specialised kernel
                    j.cp_in = T.cpk + ((size_t)b * nc + c) * T.cpk_words;
                    j.cp_stride = 1;
                    j.cp_words = T.plan->static_words;
                } else {
                    j.src = T.cp + ((size_t)b * nc + c) * nq;
                    j.raw = true;
                }
                j.t0 = meta >> 2;
            }
        } else {
            // set on every lane (the kernels branch on it wave-uniformly);
            // only active lanes write
            j.cp_meta = T.cpm;
            j.cp_base = T.cp;
            j.cp_bstride = (int64_t)nc * nq;
            j.cp_packed = T.cpk;
            j.cp_nc = nc;
            j.cp_pwords = T.cpk_words;
            if (T.t_begin > 0) j.cp_meta0 = T.cpm[c];
        }
    }
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
        const int tb = REPLAY ? J.t0 : T.t_begin;
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

// Serving slices on the specialised packed-row kernels: one task (64 chains
// of one request, one sweep range) per workgroup; chain states resume from
// and return to the request's slot.  The distances of one register class
// share a kernel that branches on the task's distance (wave-uniform), so a
// slice issues one launch per class rather than one per distance, and every
// task of a slice can run at once however few queues the device gives the
// process.  Classes: see serve_class_max.

template <int D>
__device__ __forceinline__ void serve_static_task(const ServeTask &T, uint32_t slo, uint32_t shi, uint16_t *lut_s,
                                                  uint4 *et_s)
{
    load_static_tables(T.plan, lut_s, et_s);
    const ChainJob J = serve_job(T, threadIdx.x, false);
    rows_static_core<D>(T.plan, J, T.t_begin, T.t_end, slo, shi, lut_s, et_s, 0);
}

// Occupancy of a serving class kernel: one wavefront per SIMD fewer than the
// annealing kernels of its distances where the several distances of a class,
// in one kernel, need more registers than any of them alone (measured: the
// merged kernels of d <= 15 and 17-21 spilled at the annealing kernels'
// occupancy).
constexpr int serve_class_waves(int dmax) { return dmax == 15 ? 7 : dmax == 21 ? 4 : static_waves(dmax); }

template <int DMAX, int... Ds>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(serve_class_waves(DMAX), serve_class_waves(DMAX))))
void k_serve_rows_class(const ServeTask *tasks, uint32_t slo, uint32_t shi)
{
    __shared__ uint16_t lut_s[256 * 6];
    __shared__ uint4 et_s[kStaticRanks];
    const ServeTask &T = tasks[blockIdx.x];
    const int d = (int)uni(T.plan->d);
    ((d == Ds ? serve_static_task<Ds>(T, slo, shi, lut_s, et_s) : (void)0), ...);
}

typedef void (*AnnealKernel)(AnnealArgs);
// kernels specialised to the planar lattice at odd d <= 15 (NULL otherwise),
// and the words of one chain's state they keep at its E_min (its rows,
// padded to a multiple of four)
AnnealKernel planar_rows_kernel(int d, bool plain);
int planar_state_words(int d);
// replica-exchange kernels (ladders of fixed inverse temperatures): the
// generic one (one chain per lane, state in LDS), and the packed-row ones
// specialised to the rotated lattice at odd d <= kLadderRowsMaxD (a task's
// chains inside one syndrome) and to the planar lattice at odd d <= 15 (NULL
// otherwise); the specialised ones keep each chain's rows at its first E_min
// (ladder_rows_state_words(d) words, planar_state_words(d) on the planar
// lattice)
AnnealKernel ladder_kernel(bool plain);
AnnealKernel ladder_rows_kernel(int d, bool plain);
AnnealKernel ladder_rows_kernel_large(int d, bool plain);   // d = 17 .. 31 (NULL otherwise)
AnnealKernel ladder_planar_kernel(int d, bool plain);
int ladder_rows_state_words(int d);
typedef void (*ServeKernel)(const ServeTask *, uint32_t, uint32_t);

// The specialised kernels live in several translation units (compiled in
// parallel): the annealing kernels by distance (each part returns its kernels
// for the distances it holds, else NULL), the serving kernels by class (each
// part returns the kernel of its class).
#define XZZX_STATIC_PARTS(X) X(a) X(b) X(c) X(d) X(e) X(f) X(g) X(h)
#define XZZX_DECLARE_PART(P) AnnealKernel static_rows_kernel_##P(int d, bool plain);
XZZX_STATIC_PARTS(XZZX_DECLARE_PART)
#undef XZZX_DECLARE_PART
ServeKernel serve_class_kernel_9();
ServeKernel serve_class_kernel_15();
ServeKernel serve_class_kernel_21();
ServeKernel serve_class_kernel_25();
ServeKernel serve_class_kernel_29();
ServeKernel serve_class_kernel_31();

}  // namespace xzzx
