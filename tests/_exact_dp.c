/*
 * Exact minimum energy of a coset { C0 * prod_f G_f^(x_f) } (Eqs. (18)-(20):
 * the least energy over all configurations with the syndrome of C0 in its
 * logical class), by variable elimination over the generator bits x_f in
 * face-id order -- a frontier dynamic program.  Test-side code, written
 * independently of the oracle and of the HIP library: it reads only the
 * generator tables (qubit and Pauli of each slot) and the weights.
 *
 * A qubit's weight is added once every generator touching it has been fixed;
 * a generator leaves the frontier once no unfinished qubit depends on it.
 * States are the bits of the frontier generators, held densely (cost
 * INT64_MAX = unreachable).  Exact for any lattice; memory 2^frontier.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DP_MAX_FRONTIER 24

/* fq[nstab][4]: qubit on each slot or -1; fm[nstab][4]: the generator's Pauli
 * code there (Z=1, X=2); c0[nq]: codes of the coset's base configuration;
 * w[4]: weight of each code (I, Z, X, Y).  Returns the minimum, or -1 if the
 * frontier would exceed DP_MAX_FRONTIER generators, -2 on allocation failure. */
int64_t dp_coset_minimum(int nq, int nstab, const int32_t *fq, const uint8_t *fm, const uint8_t *c0,
                         const int32_t w[4])
{
    int *last = (int *)malloc(sizeof(int) * (size_t)nq);           /* last generator touching each qubit */
    int *until = (int *)malloc(sizeof(int) * (size_t)nstab);       /* last generator needing each generator */
    int *front = (int *)malloc(sizeof(int) * (size_t)nstab);       /* frontier generator ids, bit i = front[i] */
    int64_t *cur = NULL, *nxt = NULL;
    int64_t result = -2;
    if (!last || !until || !front) goto out;
    for (int q = 0; q < nq; ++q) last[q] = -1;
    for (int f = 0; f < nstab; ++f)
        for (int s = 0; s < 4; ++s)
            if (fq[4 * f + s] >= 0 && f > last[fq[4 * f + s]]) last[fq[4 * f + s]] = f;
    for (int f = 0; f < nstab; ++f) {
        until[f] = f;
        for (int s = 0; s < 4; ++s)
            if (fq[4 * f + s] >= 0 && last[fq[4 * f + s]] > until[f]) until[f] = last[fq[4 * f + s]];
    }
    int64_t base = 0;                                 /* qubits no generator touches */
    for (int q = 0; q < nq; ++q)
        if (last[q] < 0) base += w[c0[q] & 3];
    cur = (int64_t *)malloc(sizeof(int64_t));
    if (!cur) goto out;
    cur[0] = base;
    int nf = 0;
    for (int g = 0; g < nstab; ++g) {
        /* add generator g as the frontier's top bit */
        if (nf + 1 > DP_MAX_FRONTIER) { result = -1; goto out; }
        front[nf] = g;
        const size_t n_new = (size_t)1 << (nf + 1);
        nxt = (int64_t *)malloc(sizeof(int64_t) * n_new);
        if (!nxt) goto out;
        /* qubits finished by g, and for each the frontier bits (and the
         * Pauli code) of the generators touching it */
        int nfin = 0, fin_q[4], fin_n[4], fin_bit[4][4];
        uint8_t fin_m[4][4];
        for (int s = 0; s < 4; ++s) {
            const int q = fq[4 * g + s];
            if (q < 0 || last[q] != g) continue;
            fin_q[nfin] = q;
            fin_n[nfin] = 0;
            for (int i = 0; i <= nf; ++i)
                for (int t = 0; t < 4; ++t)
                    if (fq[4 * front[i] + t] == q) {
                        fin_bit[nfin][fin_n[nfin]] = i;
                        fin_m[nfin][fin_n[nfin]++] = fm[4 * front[i] + t];
                    }
            ++nfin;
        }
        for (size_t st = 0; st < n_new; ++st) {
            const int64_t c = cur[st & (((size_t)1 << nf) - 1)];
            if (c == INT64_MAX) { nxt[st] = INT64_MAX; continue; }
            int64_t add = 0;
            for (int k = 0; k < nfin; ++k) {
                uint8_t code = c0[fin_q[k]];
                for (int j = 0; j < fin_n[k]; ++j)
                    if ((st >> fin_bit[k][j]) & 1) code ^= fin_m[k][j];
                add += w[code & 3];
            }
            nxt[st] = c + add;
        }
        free(cur);
        cur = nxt;
        nxt = NULL;
        ++nf;
        /* drop the generators no unfinished qubit needs, keeping the least cost */
        int keep[DP_MAX_FRONTIER], nk = 0;
        for (int i = 0; i < nf; ++i)
            if (until[front[i]] > g) keep[nk++] = i;
        if (nk < nf) {
            const size_t n_keep = (size_t)1 << nk;
            int64_t *red = (int64_t *)malloc(sizeof(int64_t) * n_keep);
            if (!red) goto out;
            for (size_t k = 0; k < n_keep; ++k) red[k] = INT64_MAX;
            for (size_t st = 0; st < ((size_t)1 << nf); ++st) {
                if (cur[st] == INT64_MAX) continue;
                size_t k = 0;
                for (int j = 0; j < nk; ++j) k |= ((st >> keep[j]) & 1) << j;
                if (cur[st] < red[k]) red[k] = cur[st];
            }
            int nfront[DP_MAX_FRONTIER];
            for (int j = 0; j < nk; ++j) nfront[j] = front[keep[j]];
            for (int j = 0; j < nk; ++j) front[j] = nfront[j];
            nf = nk;
            free(cur);
            cur = red;
        }
    }
    result = INT64_MAX;
    for (size_t st = 0; st < ((size_t)1 << nf); ++st)
        if (cur[st] < result) result = cur[st];
out:
    free(last); free(until); free(front); free(cur); free(nxt);
    return result;
}
