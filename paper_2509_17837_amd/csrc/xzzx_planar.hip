// Packed-row annealing kernels specialised to the planar lattice at distance
// D (odd, 3..15); the building blocks are in xzzx_planar.h.
#include "xzzx_planar.h"

namespace xzzx {

// snap: each chain's rows at its first E_min, chain-major (word i of chain ci
// at snap[ci * planar_state_words(D) + i], 16-byte aligned rows of words, so
// a lane stores them with a few wide stores from one base address), from
// which the recovery is gathered
template <int D>
__device__ __forceinline__ void planar_static_core(const PlanDev *pl, const ChainJob &J, uint32_t seed_lo,
                                                   uint32_t seed_hi, const uint16_t *lut_s, uint4 *et_s,
                                                   uint32_t *snap)
{
    using PR = PlanarRows<D>;
    const int lane = threadIdx.x;
    const int nranks = (int)uni(pl->nranks), n_sweeps = (int)uni(pl->n_sweeps), kneg = (int)uni(pl->kneg);
    int32_t W[4];
    W[0] = 0; W[1] = (int32_t)uni(pl->W[1]); W[2] = (int32_t)uni(pl->W[2]); W[3] = (int32_t)uni(pl->W[3]);
    const uint32_t uid = J.uid, cc = J.cc;
    const uint32_t k0 = uni(seed_lo), k1 = uni(seed_hi);
    const PlanarLaneKey lk = planar_lane_key(uid, k1);
    const bool use_x = J.lp == 1 || J.lp == 2, use_z = J.lp == 2 || J.lp == 3;

    uint32_t r[PR::N];
    int32_t E = planar_load<D>(pl, J, use_x, use_z, W, r);
    int32_t Emin = E, stop = 0;
    constexpr int NP = (PR::N + 3) / 4 * 4;
    uint4 *keep = (snap && J.active) ? reinterpret_cast<uint4 *>(snap + J.ci * NP) : nullptr;
    auto keep_min = [&]() { store_rows(keep, r); };
    if (keep) keep_min();
    for (int t = 0; t < n_sweeps; ++t) {
        wave_lds_fence();
        // this sweep's thresholds; 0 for the ranks with dE <= 0 (see accept_sel)
        for (int i = lane; i < nranks; i += kWave) et_s[i].y = i < kneg ? 0u : pl->thr[(size_t)t * nranks + i];
        wave_lds_fence();
        const uint32_t c2 = 4u * (uint32_t)t;
        int32_t acc = 0;
        planar_class<D, 0, planar_pipelined(D)>(r, lk, cc, c2, k0, k1, lut_s, et_s, acc);
        E += acc;
        if (E < Emin) { Emin = E; stop = 4 * t + 1; if (keep) keep_min(); }
        acc = 0;
        planar_class<D, 1, planar_pipelined(D)>(r, lk, cc, c2 + 1u, k0, k1, lut_s, et_s, acc);
        E += acc;
        if (E < Emin) { Emin = E; stop = 4 * t + 2; if (keep) keep_min(); }
        acc = 0;
        planar_class<D, 2, planar_pipelined(D)>(r, lk, cc, c2 + 2u, k0, k1, lut_s, et_s, acc);
        E += acc;
        if (E < Emin) { Emin = E; stop = 4 * t + 3; if (keep) keep_min(); }
        acc = 0;
        planar_class<D, 3, planar_pipelined(D)>(r, lk, cc, c2 + 3u, k0, k1, lut_s, et_s, acc);
        E += acc;
        if (E < Emin) { Emin = E; stop = 4 * t + 4; if (keep) keep_min(); }
    }
    if (J.active) {
        J.emin[J.ci] = Emin;
        J.stop[J.ci] = stop;
        J.efin[J.ci] = E;
        if (J.states) planar_unpack<D>(r, J.states + (size_t)J.ci * PlanarSchedule<D>::NQ);
    }
}

// MODE 0: persistent wavefronts on the atomic task queue; 2: one task per
// workgroup.  Tasks of 64 consecutive chains of a group.
template <int MODE, int D>
__device__ __forceinline__ void planar_rows_body(const AnnealArgs &A)
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
        planar_static_core<D>(G.plan, J, A.seed_lo, A.seed_hi, lut_s, et_s, G.min_snap);
    }
}

template <int D>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(planar_waves(D), planar_waves(D))))
void k_anneal_planar_d(AnnealArgs A) { planar_rows_body<0, D>(A); }
template <int D>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(planar_waves(D), planar_waves(D))))
void k_anneal_planar_d_plain(AnnealArgs A) { planar_rows_body<2, D>(A); }

int planar_state_words(int d)
{
    return ((2 * d - 1) * (2 * (2 * d + 1) <= 32 ? 1 : 2) + 3) / 4 * 4;
}

AnnealKernel planar_rows_kernel(int d, bool plain)
{
    switch (d) {
    case 3: return plain ? k_anneal_planar_d_plain<3> : k_anneal_planar_d<3>;
    case 5: return plain ? k_anneal_planar_d_plain<5> : k_anneal_planar_d<5>;
    case 7: return plain ? k_anneal_planar_d_plain<7> : k_anneal_planar_d<7>;
    case 9: return plain ? k_anneal_planar_d_plain<9> : k_anneal_planar_d<9>;
    case 11: return plain ? k_anneal_planar_d_plain<11> : k_anneal_planar_d<11>;
    case 13: return plain ? k_anneal_planar_d_plain<13> : k_anneal_planar_d<13>;
    case 15: return plain ? k_anneal_planar_d_plain<15> : k_anneal_planar_d<15>;
    default: return nullptr;
    }
}

// host-side check of the compile-time schedule against a plan's tables
template <int D>
static bool planar_matches_d(const std::vector<uint32_t> &rowface, int mpad, const std::vector<uint32_t> &qpos)
{
    constexpr const PlanarSchedule<D> &S = kPlanarSchedule<D>;
    if (mpad != PlanarSchedule<D>::MP || (int)qpos.size() != PlanarSchedule<D>::NQ) return false;
    for (int k = 0; k < 4; ++k)
        for (int m = 0; m < mpad; ++m) {
            const RotGen g = S.g[k][m];
            const uint32_t want = (uint32_t)g.Y | ((uint32_t)g.bo << 8) | ((uint32_t)g.shp << 16);
            if (rowface[k * mpad + m] != want) return false;
        }
    for (int q = 0; q < PlanarSchedule<D>::NQ; ++q)
        if (qpos[q] != S.qpos[q]) return false;
    return true;
}

bool planar_schedule_matches(int d, const std::vector<uint32_t> &rowface, int mpad, const std::vector<uint32_t> &qpos)
{
    switch (d) {
    case 3: return planar_matches_d<3>(rowface, mpad, qpos);
    case 5: return planar_matches_d<5>(rowface, mpad, qpos);
    case 7: return planar_matches_d<7>(rowface, mpad, qpos);
    case 9: return planar_matches_d<9>(rowface, mpad, qpos);
    case 11: return planar_matches_d<11>(rowface, mpad, qpos);
    case 13: return planar_matches_d<13>(rowface, mpad, qpos);
    case 15: return planar_matches_d<15>(rowface, mpad, qpos);
    default: return false;
    }
}

}  // namespace xzzx
