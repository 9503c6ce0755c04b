// Building blocks of the packed-row kernels specialised to the planar
// lattice at distance D (odd, 3..15): the lattice turned by 45 degrees (rows
// of 2D + 1 columns, see PlanarSchedule), every row in registers for the
// whole run, the generator schedule in the instruction stream.  One chain per
// lane; a task's 64 chains may span syndromes (the paper's N_SA = 10 gives 40
// chains per syndrome), so every lane draws its own Philox blocks.  Used by
// the annealing and the replica-exchange kernels of this lattice.
#pragma once

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

// The chain's starting state packed into the turned rows (the logical
// operators of its coset applied as asked), and its energy.
template <int D>
__device__ __forceinline__ int32_t planar_load(const PlanDev *pl, const ChainJob &J, bool use_x, bool use_z,
                                               const int32_t (&W)[4], uint32_t (&r)[PlanarRows<D>::N])
{
    using PR = PlanarRows<D>;
    constexpr int NW = PR::NW;
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
    return E;
}

// One byte per qubit (the lattice's qubit order) from the turned rows.
template <int D>
__device__ __forceinline__ void planar_unpack(const uint32_t (&r)[PlanarRows<D>::N], uint8_t *dst)
{
    using PR = PlanarRows<D>;
    constexpr int NW = PR::NW;
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

// The rows of a chain, stored with 16-byte stores from one base address
// (NP = the rows padded to a multiple of four words).
template <int N>
__device__ __forceinline__ void store_rows(uint4 *dst, const uint32_t (&r)[N])
{
    constexpr int NP = (N + 3) / 4 * 4;
#pragma unroll
    for (int i = 0; i < NP / 4; ++i)
        dst[i] = make_uint4(r[4 * i], 4 * i + 1 < N ? r[4 * i + 1] : 0u, 4 * i + 2 < N ? r[4 * i + 2] : 0u,
                            4 * i + 3 < N ? r[4 * i + 3] : 0u);
}

// wavefronts per SIMD (VGPR budget 512 / waves): the rows take 2D - 1
// registers (one word per row, d <= 7) or 2(2D - 1), and each lane's own
// Philox blocks take more than the split form of the rotated kernels; the
// most waves that compile without spills (at d = 9 five waves spill a few
// registers and measured 3 % slower than four)
constexpr int planar_waves(int d) { return d <= 5 ? 8 : d == 7 ? 6 : d == 9 ? 4 : d == 11 ? 4 : 3; }

}  // namespace xzzx
