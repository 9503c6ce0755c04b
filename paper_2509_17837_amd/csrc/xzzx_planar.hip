// Packed-row annealing kernels specialised to the planar lattice at distance
// D (odd, 3..15): the lattice turned by 45 degrees (rows of 2D + 1 columns,
// see PlanarSchedule), every row in registers for the whole run, the
// generator schedule in the instruction stream.  One chain per lane; a
// task's 64 chains may span syndromes (the paper's N_SA = 10 gives 40 chains
// per syndrome), so every lane draws its own Philox blocks.
#include "xzzx_device.h"

namespace xzzx {

template <int D>
struct PlanarRows {
    static constexpr int R = 2 * D - 1;                        // rows
    static constexpr int C = 2 * D + 1;                        // columns (the last two are padding)
    static constexpr int NW = 2 * C <= 32 ? 1 : 2;             // words per row
    static constexpr int N = R * NW;                           // registers per chain
};

template <int D, int K, int B, int W>
struct PlanarGen {
    static constexpr RotGen g = kPlanarSchedule<D>.g[K][4 * B + W];
    static constexpr bool real = g.shp != 5;
    static constexpr int Y = g.Y, BO = g.bo;
};

// The move's energy-table entry from its 8-bit block pattern (top row, then
// bottom row).
template <int D, int K, int B, int W>
__device__ __forceinline__ uint4 planar_lookup(const uint32_t (&r)[PlanarRows<D>::N], const uint16_t *lut_s,
                                               const uint4 *et_s)
{
    using G = PlanarGen<D, K, B, W>;
    constexpr int NW = PlanarRows<D>::NW;
    if constexpr (!G::real) {
        return make_uint4(0u, 0u, 0u, 0u);
    } else {
        const uint32_t pat2 = (row_bits<NW, G::BO, 1>(r + G::Y * NW) & 0x1Eu) |
                              (row_bits<NW, G::BO, 5>(r + (G::Y + 1) * NW) & 0x1E0u);
        const uint32_t off = *reinterpret_cast<const uint16_t *>(reinterpret_cast<const uint8_t *>(lut_s) +
                                                                 512u * G::g.shp + pat2);
        return *reinterpret_cast<const uint4 *>(reinterpret_cast<const uint8_t *>(et_s) + off);
    }
}

template <int D, int K, int B, int W>
__device__ __forceinline__ void planar_apply(uint32_t (&r)[PlanarRows<D>::N], uint32_t u, const uint4 &e, int32_t &acc)
{
    using G = PlanarGen<D, K, B, W>;
    constexpr int NW = PlanarRows<D>::NW;
    if constexpr (G::real) {
        const uint32_t sel = accept_sel(u, e.y, e.z);
        row_flip_static<NW, G::BO, 6u>(r + G::Y * NW, sel);         // X top-left | Z top-right
        row_flip_static<NW, G::BO, 9u>(r + (G::Y + 1) * NW, sel);   // Z bottom-left | X bottom-right
        acc += (int32_t)(e.x & sel);
    }
}

template <int D, int K, int B>
__device__ __forceinline__ void planar_block(uint32_t (&r)[PlanarRows<D>::N], uint32_t uid, uint32_t cc, uint32_t c2,
                                             uint32_t k0, uint32_t k1, const uint16_t *lut_s, const uint4 *et_s,
                                             int32_t &acc)
{
    const uint4 u = philox4x32_10(make_uint4(uid, cc, c2, (uint32_t)B), k0, k1);
    // the four generators of a block act on disjoint qubits: all four look up
    // their entries before any flip
    const uint4 e0 = planar_lookup<D, K, B, 0>(r, lut_s, et_s);
    const uint4 e1 = planar_lookup<D, K, B, 1>(r, lut_s, et_s);
    const uint4 e2 = planar_lookup<D, K, B, 2>(r, lut_s, et_s);
    const uint4 e3 = planar_lookup<D, K, B, 3>(r, lut_s, et_s);
    planar_apply<D, K, B, 0>(r, u.x, e0, acc);
    planar_apply<D, K, B, 1>(r, u.y, e1, acc);
    planar_apply<D, K, B, 2>(r, u.z, e2, acc);
    planar_apply<D, K, B, 3>(r, u.w, e3, acc);
    asm("" : "+v"(acc));   // sum block by block (see static_block)
}

template <int D, int K, int... Bs>
__device__ __forceinline__ void planar_class(uint32_t (&r)[PlanarRows<D>::N], uint32_t uid, uint32_t cc, uint32_t c2,
                                             uint32_t k0, uint32_t k1, const uint16_t *lut_s, const uint4 *et_s,
                                             int32_t &acc, std::integer_sequence<int, Bs...>)
{
    (planar_block<D, K, Bs>(r, uid, cc, c2, k0, k1, lut_s, et_s, acc), ...);
}

// qubit at row Y, column C of the turned lattice, or -1
template <int D>
__device__ __forceinline__ int planar_qubit_at(int Y, int C)
{
    const int u = Y + 1, v = C - (D - 1);
    return PlanarSchedule<D>::qubit(u + v + 1, u - v);
}

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
    constexpr int NW = PR::NW;
    constexpr int NB = PlanarSchedule<D>::MP / 4;
    using Blocks = std::make_integer_sequence<int, NB>;
    const int lane = threadIdx.x;
    const int nranks = (int)uni(pl->nranks), n_sweeps = (int)uni(pl->n_sweeps), kneg = (int)uni(pl->kneg);
    int32_t W[4];
    W[0] = 0; W[1] = (int32_t)uni(pl->W[1]); W[2] = (int32_t)uni(pl->W[2]); W[3] = (int32_t)uni(pl->W[3]);
    const uint32_t uid = J.uid, cc = J.cc;
    const uint32_t k0 = uni(seed_lo), k1 = uni(seed_hi);
    const bool use_x = J.lp == 1 || J.lp == 2, use_z = J.lp == 2 || J.lp == 3;

    uint32_t r[PR::N];
    int32_t E = 0;
#pragma unroll
    for (int Y = 0; Y < PR::R; ++Y) {
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            uint32_t word = 0;
            if (J.active) {
#pragma unroll 1
                for (int C = 16 * w; C < min(PR::C, 16 * w + 16); ++C) {
                    const int q = planar_qubit_at<D>(Y, C);
                    if (q < 0) continue;
                    uint32_t v = J.src[q] & 3u;
                    if (use_x) v ^= pl->lx[q];
                    if (use_z) v ^= pl->lz[q];
                    word |= v << (2 * (C - 16 * w));
                    E += weight_of(W, v);
                }
            }
            r[Y * NW + w] = word;
        }
    }
    int32_t Emin = E, stop = 0;
    constexpr int NP = (PR::N + 3) / 4 * 4;
    uint4 *keep = (snap && J.active) ? reinterpret_cast<uint4 *>(snap + J.ci * NP) : nullptr;
    auto keep_min = [&]() {
#pragma unroll
        for (int i = 0; i < NP / 4; ++i)
            keep[i] = make_uint4(r[4 * i], 4 * i + 1 < PR::N ? r[4 * i + 1] : 0u, 4 * i + 2 < PR::N ? r[4 * i + 2] : 0u,
                                 4 * i + 3 < PR::N ? r[4 * i + 3] : 0u);
    };
    if (keep) keep_min();
    for (int t = 0; t < n_sweeps; ++t) {
        wave_lds_fence();
        // this sweep's thresholds; 0 for the ranks with dE <= 0 (see accept_sel)
        for (int i = lane; i < nranks; i += kWave) et_s[i].y = i < kneg ? 0u : pl->thr[(size_t)t * nranks + i];
        wave_lds_fence();
        const uint32_t c2 = 4u * (uint32_t)t;
        int32_t acc = 0;
        planar_class<D, 0>(r, uid, cc, c2, k0, k1, lut_s, et_s, acc, Blocks{});
        E += acc;
        if (E < Emin) { Emin = E; stop = 4 * t + 1; if (keep) keep_min(); }
        acc = 0;
        planar_class<D, 1>(r, uid, cc, c2 + 1u, k0, k1, lut_s, et_s, acc, Blocks{});
        E += acc;
        if (E < Emin) { Emin = E; stop = 4 * t + 2; if (keep) keep_min(); }
        acc = 0;
        planar_class<D, 2>(r, uid, cc, c2 + 2u, k0, k1, lut_s, et_s, acc, Blocks{});
        E += acc;
        if (E < Emin) { Emin = E; stop = 4 * t + 3; if (keep) keep_min(); }
        acc = 0;
        planar_class<D, 3>(r, uid, cc, c2 + 3u, k0, k1, lut_s, et_s, acc, Blocks{});
        E += acc;
        if (E < Emin) { Emin = E; stop = 4 * t + 4; if (keep) keep_min(); }
    }
    if (J.active) {
        J.emin[J.ci] = Emin;
        J.stop[J.ci] = stop;
        J.efin[J.ci] = E;
        if (J.states) {
            uint8_t *dst = J.states + (size_t)J.ci * PlanarSchedule<D>::NQ;
#pragma unroll
            for (int Y = 0; Y < PR::R; ++Y)
#pragma unroll
                for (int w = 0; w < NW; ++w)
#pragma unroll 1
                    for (int C = 16 * w; C < min(PR::C, 16 * w + 16); ++C) {
                        const int q = planar_qubit_at<D>(Y, C);
                        if (q >= 0) dst[q] = (uint8_t)((r[Y * NW + w] >> (2 * (C - 16 * w))) & 3u);
                    }
        }
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

// wavefronts per SIMD (VGPR budget 512 / waves): the rows take 2D - 1
// registers (one word per row, d <= 7) or 2(2D - 1), and each lane's own
// Philox blocks take more than the split form of the rotated kernels; the
// most waves that compile without spills (at d = 9 five waves spill a few
// registers and measured 3 % slower than four)
constexpr int planar_waves(int d) { return d <= 5 ? 8 : d == 7 ? 6 : d == 9 ? 4 : d == 11 ? 4 : 3; }

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
