// Replica exchange (parallel tempering) on ladders of fixed inverse
// temperatures: one chain per lane, colour-class sweeps at the chain's level,
// then exchanges of adjacent levels between the chains of a ladder.
//
// A group's replicas come in ladders of K consecutive replicas, so the chains
// 4(bK + j) + P, j = 0..K-1, of coset P of ladder b sit in the lanes
// P, P + 4, ..., P + 4(K - 1) of one aligned block of 4K lanes (a task of 64
// consecutive chains holds whole blocks: 4K divides 64 and 4 n_rep).  The
// state of chain c is packed 2 bits per qubit, word w at LDS word 64 w + c
// (all lanes move the same generator at once, so each access is 64
// consecutive words); position nq is scratch for absent generator slots.
#include "xzzx_device.h"

namespace xzzx {

struct LadderLds {
    uint32_t desc, lut, et, state, e, pos;
};

__device__ __forceinline__ LadderLds ladder_layout(int M, int ntypes, int nranks, int K, int nq)
{
    LadderLds o;
    o.desc = 0;
    o.lut = 8u * 4u * (uint32_t)M;
    o.et = (o.lut + 256u * (uint32_t)ntypes + 7u) & ~7u;
    o.state = (o.et + 8u * (uint32_t)nranks * (uint32_t)K + 15u) & ~15u;
    o.e = o.state + 4u * (uint32_t)(nq / 16 + 1) * kWave;
    o.pos = o.e + 4u * kWave;
    return o;
}

// snap: each chain's packed state at its first E_min (word w of chain ci at
// snap[w * snap_stride + ci]), from which the recovery is gathered
__device__ inline void ladder_core(const PlanDev *pl, const ChainJob &J, uint32_t seed_lo, uint32_t seed_hi,
                                   uint8_t *smem, uint32_t *snap, int64_t snap_stride)
{
    const int lane = threadIdx.x;
    const int nq = pl->nq, M = pl->M, nblk = pl->nblk, nranks = pl->nranks, n_sweeps = pl->n_sweeps;
    const int K = pl->ladder_k;
    const uint32_t kneg = (uint32_t)pl->kneg;
    int32_t W[4];
    W[0] = pl->W[0]; W[1] = pl->W[1]; W[2] = pl->W[2]; W[3] = pl->W[3];
    const LadderLds lo = ladder_layout(M, pl->ntypes, nranks, K, nq);
    const uint2 *desc_s = reinterpret_cast<const uint2 *>(smem + lo.desc);
    const uint8_t *lut_s = smem + lo.lut;
    const int2 *et_s = reinterpret_cast<const int2 *>(smem + lo.et);
    uint32_t *st = reinterpret_cast<uint32_t *>(smem + lo.state);
    int32_t *e_s = reinterpret_cast<int32_t *>(smem + lo.e);
    int32_t *pos_s = reinterpret_cast<int32_t *>(smem + lo.pos);
    const int nw = nq / 16 + 1;
    const uint32_t uid = J.uid, cc = J.cc;
    // ladder position: replica r = bK + j, coset P; block of 4K lanes
    const uint32_t rep = cc >> 2, P = cc & 3u;
    const int j = (int)(rep % (uint32_t)K);
    const uint32_t ladder_id = 4u * (rep / (uint32_t)K) + P;
    const int base = lane & ~(4 * K - 1);
    int level = j;

    const bool use_x = (J.lp == 1 || J.lp == 2), use_z = (J.lp == 2 || J.lp == 3);
    int32_t E = 0;
    for (int w = 0; w < nw; ++w) {
        uint32_t word = 0;
        for (int i = 0; i < 16; ++i) {
            const int q = 16 * w + i;
            if (q >= nq) break;
            uint32_t v = J.active ? (J.src[q] & 3u) : 0u;
            if (J.active && use_x) v ^= pl->lx[q];
            if (J.active && use_z) v ^= pl->lz[q];
            word |= v << (2 * i);
            E += weight_of(W, v);
        }
        st[w * kWave + lane] = word;
    }
    int32_t Emin = E, stop = 0;
    const bool keep = snap != nullptr && J.active;
    auto keep_min = [&]() {
        for (int w = 0; w < nw; ++w) snap[(int64_t)w * snap_stride + J.ci] = st[w * kWave + lane];
    };
    if (keep) keep_min();
    wave_lds_fence();

    for (int t = 0; t < n_sweeps; ++t) {
        const int2 *et_l = et_s + level * nranks;
        for (int k = 0; k < 4; ++k) {
            const uint2 *dk = desc_s + k * M;
            int32_t acc = 0;
            for (int b = 0; b < nblk; ++b) {
                const uint4 rnd = philox4x32_10(make_uint4(uid, cc, 4u * (uint32_t)t + (uint32_t)k, (uint32_t)b),
                                                seed_lo, seed_hi);
                const uint32_t uw[4] = {rnd.x, rnd.y, rnd.z, rnd.w};
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    if (4 * b + g >= M) break;
                    const uint2 d = dk[4 * b + g];
                    const uint32_t q0 = d.x & 0xFFFFu, q1 = d.x >> 16, q2 = d.y & 0xFFFFu, q3 = (d.y >> 16) & 0x7FFu;
                    uint32_t *a0 = st + (q0 >> 4) * kWave + lane, *a1 = st + (q1 >> 4) * kWave + lane;
                    uint32_t *a2 = st + (q2 >> 4) * kWave + lane, *a3 = st + (q3 >> 4) * kWave + lane;
                    const uint32_t s0 = 2u * (q0 & 15u), s1 = 2u * (q1 & 15u), s2 = 2u * (q2 & 15u),
                                   s3 = 2u * (q3 & 15u);
                    const uint32_t pat = ((*a0 >> s0) & 3u) | (((*a1 >> s1) & 3u) << 2) |
                                         (((*a2 >> s2) & 3u) << 4) | (((*a3 >> s3) & 3u) << 6);
                    const uint32_t rank = lut_s[((d.y >> 27) << 8) | pat];
                    const int2 et = et_l[rank];
                    if (rank < kneg || uw[g] < (uint32_t)et.y) {
                        // slots 0 and 3 carry X, 1 and 2 carry Z; slots may share a word
                        *a0 ^= 2u << s0;
                        *a1 ^= 1u << s1;
                        *a2 ^= 1u << s2;
                        *a3 ^= 2u << s3;
                        acc += et.x;
                    }
                }
            }
            E += acc;
            if (E < Emin) {
                Emin = E;
                stop = 4 * t + k + 1;
                if (keep) keep_min();
            }
        }
        // exchanges between levels (k, k + 1), k = t mod 2, t mod 2 + 2, ...
        if (K > 1) {
            e_s[lane] = E;
            pos_s[base + 4 * level + (int)P] = lane;
            wave_lds_fence();
            const int par = t & 1;
            const bool low = ((level - par) & 1) == 0;
            const int plevel = low ? level + 1 : level - 1;
            if (plevel >= 0 && plevel < K) {
                const int partner = pos_s[base + 4 * plevel + (int)P];
                const int32_t e_lo = low ? E : e_s[partner], e_hi = low ? e_s[partner] : E;
                const int kp = low ? level : plevel;
                const uint32_t p = (uint32_t)(kp - par) >> 1;
                const uint4 rr = philox4x32_10(make_uint4(uid, 0x80000000u | ladder_id, (uint32_t)t, p >> 2),
                                               seed_lo, seed_hi);
                const uint32_t uws[4] = {rr.x, rr.y, rr.z, rr.w};
                const uint32_t u = uws[p & 3u];
                if (e_hi >= e_lo || u < swap_threshold(pl->ladder_pow, (uint32_t)(e_lo - e_hi))) level = plevel;
            }
            wave_lds_fence();
        }
    }
    if (J.active) {
        J.emin[J.ci] = Emin;
        J.stop[J.ci] = stop;
        J.efin[J.ci] = E;
        if (J.states) {
            uint8_t *dst = J.states + (size_t)J.ci * nq;
            for (int q = 0; q < nq; ++q) dst[q] = (uint8_t)((st[(q >> 4) * kWave + lane] >> (2 * (q & 15))) & 3u);
        }
    }
    wave_lds_fence();
}

// MODE 0: persistent wavefronts on the atomic task queue; 2: one task per
// workgroup.  Tasks of 64 consecutive chains of a group.
template <int MODE>
__device__ __forceinline__ void ladder_body(const AnnealArgs &A)
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
        const PlanDev *pl = G.plan;
        if (pl != loaded) {
            wave_lds_fence();
            const LadderLds lo = ladder_layout(pl->M, pl->ntypes, pl->nranks, pl->ladder_k, pl->nq);
            uint2 *desc_s = reinterpret_cast<uint2 *>(smem + lo.desc);
            for (int i = threadIdx.x; i < 4 * pl->M; i += kWave) desc_s[i] = reinterpret_cast<const uint2 *>(pl->desc)[i];
            uint32_t *lut_s = reinterpret_cast<uint32_t *>(smem + lo.lut);
            for (int i = threadIdx.x; i < 64 * pl->ntypes; i += kWave) lut_s[i] = reinterpret_cast<const uint32_t *>(pl->lut)[i];
            int2 *et_s = reinterpret_cast<int2 *>(smem + lo.et);
            for (int i = threadIdx.x; i < pl->ladder_k * pl->nranks; i += kWave)
                et_s[i] = make_int2(pl->dE[i % pl->nranks], (int)pl->ladder_thr[i]);
            wave_lds_fence();
            loaded = pl;
        }
        const ChainJob J = batch_job(G, unit0 + threadIdx.x, false);
        ladder_core(pl, J, A.seed_lo, A.seed_hi, smem, G.min_snap, G.n_chains);
    }
}

__global__ __launch_bounds__(kWave) void k_anneal_ladder(AnnealArgs A) { ladder_body<0>(A); }
__global__ __launch_bounds__(kWave) void k_anneal_ladder_plain(AnnealArgs A) { ladder_body<2>(A); }

AnnealKernel ladder_kernel(bool plain) { return plain ? k_anneal_ladder_plain : k_anneal_ladder; }

}  // namespace xzzx
