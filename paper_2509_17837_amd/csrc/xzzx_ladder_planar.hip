// Replica exchange on the packed-row kernels specialised to the planar
// lattice at distance D (odd, 3..15): the annealing kernel's sweep (turned
// rows in registers, compile-time schedule, each lane its own Philox
// blocks), with each lane's move entries read from the table of its chain's
// current level, an exchange of adjacent levels after every sweep, and each
// chain's rows kept at its first E_min.  Chains, draws and exchanges are
// those of the generic ladder kernel, bit for bit.
#include "xzzx_planar.h"

namespace xzzx {

// snap: each chain's rows at its first E_min, chain-major (word i of chain
// ci at snap[ci * planar_state_words(D) + i])
template <int D>
__device__ __forceinline__ void ladder_planar_core(const PlanDev *pl, const ChainJob &J, uint32_t seed_lo,
                                                   uint32_t seed_hi, const uint16_t *lut_s, const uint4 *et_s,
                                                   uint32_t *snap)
{
    using PR = PlanarRows<D>;
    const int nranks = (int)uni(pl->nranks), n_sweeps = (int)uni(pl->n_sweeps), K = (int)uni(pl->ladder_k);
    int32_t W[4];
    W[0] = 0; W[1] = (int32_t)uni(pl->W[1]); W[2] = (int32_t)uni(pl->W[2]); W[3] = (int32_t)uni(pl->W[3]);
    const uint32_t uid = J.uid, cc = J.cc;
    const uint32_t k0 = uni(seed_lo), k1 = uni(seed_hi);
    const PlanarLaneKey lk = planar_lane_key(uid, k1);
    // ladder position: replica r = bK + j starts at level j; coset P
    const uint32_t rep = cc >> 2, P = cc & 3u;
    const uint32_t ladder_id = 4u * (rep / (uint32_t)K) + P;
    int level = (int)(rep % (uint32_t)K);

    uint32_t r[PR::N];
    int32_t E = planar_load<D>(pl, J, J.lp == 1 || J.lp == 2, J.lp == 2 || J.lp == 3, W, r);
    int32_t Emin = E, stop = 0;
    constexpr int NP = (PR::N + 3) / 4 * 4;
    uint4 *keep = (snap && J.active) ? reinterpret_cast<uint4 *>(snap + J.ci * NP) : nullptr;
    if (keep) store_rows(keep, r);
    for (int t = 0; t < n_sweeps; ++t) {
        const uint4 *et_l = et_s + level * nranks;
        const uint32_t c2 = 4u * (uint32_t)t;
        int32_t acc = 0;
        planar_class<D, 0, planar_ladder_pipelined(D)>(r, lk, cc, c2, k0, k1, lut_s, et_l, acc);
        E += acc;
        if (E < Emin) { Emin = E; stop = 4 * t + 1; if (keep) store_rows(keep, r); }
        acc = 0;
        planar_class<D, 1, planar_ladder_pipelined(D)>(r, lk, cc, c2 + 1u, k0, k1, lut_s, et_l, acc);
        E += acc;
        if (E < Emin) { Emin = E; stop = 4 * t + 2; if (keep) store_rows(keep, r); }
        acc = 0;
        planar_class<D, 2, planar_ladder_pipelined(D)>(r, lk, cc, c2 + 2u, k0, k1, lut_s, et_l, acc);
        E += acc;
        if (E < Emin) { Emin = E; stop = 4 * t + 3; if (keep) store_rows(keep, r); }
        acc = 0;
        planar_class<D, 3, planar_ladder_pipelined(D)>(r, lk, cc, c2 + 3u, k0, k1, lut_s, et_l, acc);
        E += acc;
        if (E < Emin) { Emin = E; stop = 4 * t + 4; if (keep) store_rows(keep, r); }
        if (K > 1) level = ladder_exchange(level, E, K, P, uid, ladder_id, t, k0, k1, pl->ladder_pow);
    }
    if (J.active) {
        J.emin[J.ci] = Emin;
        J.stop[J.ci] = stop;
        J.efin[J.ci] = E;
        if (J.states) planar_unpack<D>(r, J.states + (size_t)J.ci * PlanarSchedule<D>::NQ);
    }
}

template <int MODE, int D>
__device__ __forceinline__ void ladder_planar_body(const AnnealArgs &A)
{
    ladder_static_body<MODE>(A, [&](const GroupArgs &G, const ChainJob &J, const uint16_t *lut_s, const uint4 *et_s) {
        ladder_planar_core<D>(G.plan, J, A.seed_lo, A.seed_hi, lut_s, et_s, G.min_snap);
    });
}

template <int D>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(planar_waves(D), planar_waves(D))))
void k_anneal_ladder_planar_d(AnnealArgs A) { ladder_planar_body<0, D>(A); }
template <int D>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(planar_waves(D), planar_waves(D))))
void k_anneal_ladder_planar_d_plain(AnnealArgs A) { ladder_planar_body<2, D>(A); }

AnnealKernel ladder_planar_kernel(int d, bool plain)
{
    switch (d) {
    case 3: return plain ? k_anneal_ladder_planar_d_plain<3> : k_anneal_ladder_planar_d<3>;
    case 5: return plain ? k_anneal_ladder_planar_d_plain<5> : k_anneal_ladder_planar_d<5>;
    case 7: return plain ? k_anneal_ladder_planar_d_plain<7> : k_anneal_ladder_planar_d<7>;
    case 9: return plain ? k_anneal_ladder_planar_d_plain<9> : k_anneal_ladder_planar_d<9>;
    case 11: return plain ? k_anneal_ladder_planar_d_plain<11> : k_anneal_ladder_planar_d<11>;
    case 13: return plain ? k_anneal_ladder_planar_d_plain<13> : k_anneal_ladder_planar_d<13>;
    case 15: return plain ? k_anneal_ladder_planar_d_plain<15> : k_anneal_ladder_planar_d<15>;
    default: return nullptr;
    }
}

}  // namespace xzzx
