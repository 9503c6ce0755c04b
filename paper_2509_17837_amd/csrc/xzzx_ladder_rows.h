// Replica exchange on the packed-row kernels specialised to the rotated
// lattice at distance D (odd, D <= kLadderRowsMaxD).  The sweep is the
// annealing kernel's: the chain's rows stay in registers and the generator
// schedule is compile-time.  What changes: each lane reads its move entries
// from the table of its chain's current level (the levels' thresholds are
// fixed for the run, so no table is refreshed between sweeps), adjacent
// levels of a ladder try an exchange after every sweep, and each chain keeps
// its rows at its first E_min for the recovery.  Chains, draws and exchanges
// are those of the generic ladder kernel, bit for bit.
//
// A task's 64 chains lie inside one syndrome (4 n_rep is a multiple of 64),
// so the Philox counter's uid is uniform and the split form of the
// annealing kernel applies.  The kernels are instantiated over several
// translation units (xzzx_ladder_rows*.hip), which build in parallel.
#pragma once

#include "xzzx_device.h"
#include "xzzx_planar.h"

namespace xzzx {

// snap: each chain's rows at its first E_min, chain-major (word i of chain
// ci at snap[ci * ladder_rows_state_words(D) + i])
template <int D>
__device__ __forceinline__ void ladder_rows_core(const PlanDev *pl, const ChainJob &J, uint32_t seed_lo,
                                                 uint32_t seed_hi, const uint16_t *lut_s, const uint4 *et_s,
                                                 uint32_t *snap)
{
    constexpr int N = StaticRows<D>::N;
    constexpr int NB = RotSchedule<D>::MP / 4;
    using Blocks = std::make_integer_sequence<int, NB>;
    const int nranks = (int)uni(pl->nranks), n_sweeps = (int)uni(pl->n_sweeps), K = (int)uni(pl->ladder_k);
    int32_t W[4];
    W[0] = 0; W[1] = (int32_t)uni(pl->W[1]); W[2] = (int32_t)uni(pl->W[2]); W[3] = (int32_t)uni(pl->W[3]);
    const uint32_t uid = uni(J.uid), cc = J.cc;
    const uint32_t k0 = uni(seed_lo), k1 = uni(seed_hi);
    // ladder position: replica r = bK + j starts at level j; coset P
    const uint32_t rep = cc >> 2, P = cc & 3u;
    const uint32_t ladder_id = 4u * (rep / (uint32_t)K) + P;
    int level = (int)(rep % (uint32_t)K);

    uint32_t r[N];
    int32_t E = static_load<D>(pl, J, J.lp == 1 || J.lp == 2, J.lp == 2 || J.lp == 3, W, r);
    int32_t Emin = E, stop = 0;
    constexpr int NP = (N + 3) / 4 * 4;
    uint4 *keep = (snap && J.active) ? reinterpret_cast<uint4 *>(snap + J.ci * NP) : nullptr;
    if (keep) store_rows(keep, r);
    for (int t = 0; t < n_sweeps; ++t) {
        const uint4 *et_l = et_s + level * nranks;
        const uint32_t c2 = 4u * (uint32_t)t;
        int32_t acc = 0;
        static_class<D, 0>(r, philox_head(uid, cc, c2, k0, k1), k0, k1, lut_s, et_l, acc, Blocks{});
        E += acc;
        if (E < Emin) { Emin = E; stop = 4 * t + 1; if (keep) store_rows(keep, r); }
        acc = 0;
        static_class<D, 1>(r, philox_head(uid, cc, c2 + 1u, k0, k1), k0, k1, lut_s, et_l, acc, Blocks{});
        E += acc;
        if (E < Emin) { Emin = E; stop = 4 * t + 2; if (keep) store_rows(keep, r); }
        acc = 0;
        static_class<D, 2>(r, philox_head(uid, cc, c2 + 2u, k0, k1), k0, k1, lut_s, et_l, acc, Blocks{});
        E += acc;
        if (E < Emin) { Emin = E; stop = 4 * t + 3; if (keep) store_rows(keep, r); }
        acc = 0;
        static_class<D, 3>(r, philox_head(uid, cc, c2 + 3u, k0, k1), k0, k1, lut_s, et_l, acc, Blocks{});
        E += acc;
        if (E < Emin) { Emin = E; stop = 4 * t + 4; if (keep) store_rows(keep, r); }
        if (K > 1) level = ladder_exchange(level, E, K, P, uid, ladder_id, t, k0, k1, pl->ladder_pow);
    }
    if (J.active) {
        J.emin[J.ci] = Emin;
        J.stop[J.ci] = stop;
        J.efin[J.ci] = E;
        if (J.states) static_unpack<D>(r, J.states + (size_t)J.ci * (D * D));
    }
}

template <int MODE, int D>
__device__ __forceinline__ void ladder_rows_body(const AnnealArgs &A)
{
    ladder_static_body<MODE>(A, [&](const GroupArgs &G, const ChainJob &J, const uint16_t *lut_s, const uint4 *et_s) {
        ladder_rows_core<D>(G.plan, J, A.seed_lo, A.seed_hi, lut_s, et_s, G.min_snap);
    });
}

template <int D>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(static_waves(D), static_waves(D))))
void k_anneal_ladder_rows_d(AnnealArgs A) { ladder_rows_body<0, D>(A); }
template <int D>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(static_waves(D), static_waves(D))))
void k_anneal_ladder_rows_d_plain(AnnealArgs A) { ladder_rows_body<2, D>(A); }

}  // namespace xzzx
