/*
 * perc_oracle.c -- plain, slow, CPU-only reference ("oracle") for the percolation
 * inspection of Xu, Xu & Yakobson, "Site-percolation threshold of carbon nanotube
 * fibers -- fast inspection of percolation with Markov stochastic theory".
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library. It shares no code, header, table or helper
 * with the HIP product path, and the product never calls it.
 *
 * Everything is FP64 and written for a reader who checks it against the paper:
 *
 *   lattice   -- built from geometry (Sec. II.A, Fig. 1): FCC stacked along [111]
 *                (ABC layers), every site a tube along the stacking axis; two sites
 *                are side-contact neighbours when their FCC distance is the nearest-
 *                neighbour distance, end-contact neighbours when they sit in the same
 *                column three layers apart (the next tube along the axis). No offset
 *                table is used: every candidate pair in a small box is tested with the
 *                distance predicate.
 *   sampler   -- Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11), written from the
 *                published round function; Bernoulli(p) per site (Sec. II.A, <N_m>=Np).
 *                Pinned by the generator's published known-answer outputs, uniformity
 *                tests, host/device equality and a key-schedule shift identity against
 *                the closed forms of the Weyl increments.
 *   markov    -- the transition matrix of Eq. (2) built explicitly in CSR over the
 *                metallic sites plus the detector site j1 joined to every metallic site
 *                of the far end surface (Sec. II.B); forward power iteration x <- x P
 *                with the detector absorbing, plus the exact Boolean support of the
 *                iterate ("non-zero probability", Sec. II.B) which makes the decision.
 *   eq3       -- the backward first-passage recursion of Eq. (3)-(4) on an arbitrary
 *                row-stochastic CSR matrix (used for the Fig. 2 pin and to tie the
 *                forward form to the printed recursion).
 *   bfs / uf  -- the plain definition the iteration reaches exactly: is there a path of
 *                metallic neighbours from the start surface to the far surface
 *                (Sec. II.B: "equivalent to the possibility of reaching one side ...
 *                from the other" -- restated, not quoted). Breadth-first search and a
 *                union-find are independent pins.
 *   exhaust  -- all 2^N configurations of a tiny lattice: exact percolating counts a_k
 *                per number k of metallic sites, so Pi(p) = sum_k a_k p^k (1-p)^(N-k).
 *
 * Readings where the paper is silent (documented with the design notes of the
 * repository): W counts projected tube spacings and the cross-section is the hexagon
 * of that hex radius; L counts (111) layers; the start surface is the terminal tube of
 * every column at the low end (layers 0..2) and the far surface the terminal tube at
 * the high end (layers L-3..L-1); deg(i) counts metallic neighbours plus the detector
 * edge; an isolated metallic site keeps its mass (self-loop, Sec. II.B remark); the
 * mass starts uniform over the metallic start sites.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ECAP (-6) /* the N_max cap of Sec. II.B was reached: must never happen */

/* ------------------------------------------------------------------------------ */
/* Lattice from geometry (Sec. II.A, Fig. 1)                                      */
/* ------------------------------------------------------------------------------ */

typedef struct {
    int W, L;
    int64_t n;          /* number of sites */
    int32_t *q, *r, *k; /* coordinates, canonical order = lexicographic (k, q, r) */
    int64_t *nb_ptr;    /* neighbour lists, CSR, ascending site index */
    int32_t *nb;
    int64_t n_bonds;    /* undirected bonds of the full lattice */
    uint8_t *is_start;  /* k <= 2 */
    uint8_t *is_far;    /* k >= L-3 */
} orc_lattice;

static int hexdist(int q, int r) {
    int a = abs(q), b = abs(r), c = abs(q + r);
    int m = a > b ? a : b;
    return m > c ? m : c;
}

/* Column (q,r) in axial coordinates of the projected triangular net with spacing d.
 * The (111) layers of FCC are triangular nets of spacing sqrt(3) d stacked A,B,C;
 * the column (q,r) carries layers k with k == (q - r) mod 3. With the layer spacing
 * sqrt(2) d, 4 |dx|^2 / d^2 = (2dq + dr)^2 + 3 dr^2 + 8 dk^2, and the FCC nearest-
 * neighbour distance sqrt(3) d gives the value 12. */
static int mod3(int v) { int m = v % 3; return m < 0 ? m + 3 : m; }

static int is_side_contact(int dq, int dr, int dk) {
    int a = 2 * dq + dr;
    return a * a + 3 * dr * dr + 8 * dk * dk == 12;
}
static int is_end_contact(int dq, int dr, int dk) {
    return dq == 0 && dr == 0 && (dk == 3 || dk == -3);
}

void orc_lattice_free(orc_lattice *lat) {
    if (!lat) return;
    free(lat->q); free(lat->r); free(lat->k);
    free(lat->nb_ptr); free(lat->nb);
    free(lat->is_start); free(lat->is_far);
    free(lat);
}

/* ends = 1: the modified lattice of the paper (12 side + 2 end contacts); ends = 0:
 * the regular FCC lattice of the same sites (12 side contacts only), the reference
 * lattice the paper compares its threshold with (Sec. III). Surfaces are the same. */
orc_lattice *orc_lattice_new_ex(int W, int L, int ends) {
    /* L < 2^16 and W <= 1024: the Philox stream tag W<<16 | L names one shape only */
    if (W < 0 || L < 1 || W > 1024 || L > 65535) return NULL;
    orc_lattice *lat = (orc_lattice *)calloc(1, sizeof(orc_lattice));
    if (!lat) return NULL;
    lat->W = W; lat->L = L;
    /* count sites: every (q,r,k) inside the hexagon with k == (q-r) mod 3 */
    int64_t n = 0;
    for (int k = 0; k < L; ++k)
        for (int q = -W; q <= W; ++q)
            for (int r = -W; r <= W; ++r)
                if (hexdist(q, r) <= W && mod3(q - r) == mod3(k)) ++n;
    lat->n = n;
    lat->q = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    lat->r = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    lat->k = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    lat->is_start = (uint8_t *)calloc((size_t)(n ? n : 1), 1);
    lat->is_far = (uint8_t *)calloc((size_t)(n ? n : 1), 1);
    /* dense index over the bounding box so that candidate pairs are found quickly */
    int S = 2 * W + 1;
    int64_t box = (int64_t)S * S * L;
    int64_t *index = (int64_t *)malloc(sizeof(int64_t) * (size_t)box);
    if (!lat->q || !lat->r || !lat->k || !lat->is_start || !lat->is_far || !index) {
        free(index); orc_lattice_free(lat); return NULL;
    }
    for (int64_t i = 0; i < box; ++i) index[i] = -1;
    /* enumeration in (k, q, r) lexicographic order IS the canonical order */
    int64_t s = 0;
    for (int k = 0; k < L; ++k)
        for (int q = -W; q <= W; ++q)
            for (int r = -W; r <= W; ++r)
                if (hexdist(q, r) <= W && mod3(q - r) == mod3(k)) {
                    lat->q[s] = q; lat->r[s] = r; lat->k[s] = k;
                    lat->is_start[s] = (k <= 2);
                    lat->is_far[s] = (k >= L - 3);
                    index[((int64_t)k * S + (q + W)) * S + (r + W)] = s;
                    ++s;
                }
    /* neighbours: test every point of the box |dq|,|dr| <= 2, |dk| <= 3 */
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) { free(index); orc_lattice_free(lat); return NULL; }
    for (int pass = 0; pass < 2; ++pass) {
        for (int64_t i = 0; i < n; ++i) {
            int q = lat->q[i], r = lat->r[i], k = lat->k[i];
            int64_t pos = pass ? lat->nb_ptr[i] : 0;
            /* collect in ascending site index: dk outer, then q, then r */
            for (int dk = -3; dk <= 3; ++dk)
                for (int dq = -2; dq <= 2; ++dq)
                    for (int dr = -2; dr <= 2; ++dr) {
                        if (!is_side_contact(dq, dr, dk) && !(ends && is_end_contact(dq, dr, dk))) continue;
                        int q2 = q + dq, r2 = r + dr, k2 = k + dk;
                        if (k2 < 0 || k2 >= L || hexdist(q2, r2) > W) continue;
                        int64_t j = index[((int64_t)k2 * S + (q2 + W)) * S + (r2 + W)];
                        if (j < 0) continue; /* no site at that point (wrong sublattice) */
                        if (pass) lat->nb[pos++] = (int32_t)j;
                        else cnt[i]++;
                    }
        }
        if (!pass) {
            lat->nb_ptr = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
            if (!lat->nb_ptr) { free(cnt); free(index); orc_lattice_free(lat); return NULL; }
            lat->nb_ptr[0] = 0;
            for (int64_t i = 0; i < n; ++i) lat->nb_ptr[i + 1] = lat->nb_ptr[i] + cnt[i];
            lat->nb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(lat->nb_ptr[n] ? lat->nb_ptr[n] : 1));
            if (!lat->nb) { free(cnt); free(index); orc_lattice_free(lat); return NULL; }
        }
    }
    lat->n_bonds = lat->nb_ptr[n] / 2;
    free(cnt);
    free(index);
    return lat;
}

orc_lattice *orc_lattice_new(int W, int L) { return orc_lattice_new_ex(W, L, 1); }

int64_t orc_lattice_sites(const orc_lattice *lat) { return lat->n; }
int64_t orc_lattice_bonds(const orc_lattice *lat) { return lat->n_bonds; }
int64_t orc_lattice_nnz(const orc_lattice *lat) { return lat->nb_ptr[lat->n]; }

void orc_lattice_coords(const orc_lattice *lat, int32_t *q, int32_t *r, int32_t *k) {
    memcpy(q, lat->q, sizeof(int32_t) * (size_t)lat->n);
    memcpy(r, lat->r, sizeof(int32_t) * (size_t)lat->n);
    memcpy(k, lat->k, sizeof(int32_t) * (size_t)lat->n);
}

void orc_lattice_adjacency(const orc_lattice *lat, int64_t *ptr, int32_t *idx) {
    memcpy(ptr, lat->nb_ptr, sizeof(int64_t) * ((size_t)lat->n + 1));
    memcpy(idx, lat->nb, sizeof(int32_t) * (size_t)lat->nb_ptr[lat->n]);
}

void orc_lattice_surfaces(const orc_lattice *lat, uint8_t *start, uint8_t *far) {
    memcpy(start, lat->is_start, (size_t)lat->n);
    memcpy(far, lat->is_far, (size_t)lat->n);
}

/* ------------------------------------------------------------------------------ */
/* Philox4x32-10 and the Bernoulli occupancy (Sec. II.A)                           */
/* ------------------------------------------------------------------------------ */

/* One Philox round: the two 32x32 -> 64-bit products of counter words 0 and 2 by the
 * round multipliers; each high half is mixed with the other counter word and a key
 * word. Constants as published by Salmon et al. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Threshold of the integer Bernoulli rule: a site is metallic iff its uniform 32-bit
 * draw u satisfies u < floor(p * 2^32); p = 1 gives 2^32 (always), p = 0 gives 0. */
uint64_t orc_threshold(double p) {
    if (!(p >= 0.0)) return 0;
    if (p >= 1.0) return (uint64_t)1 << 32;
    return (uint64_t)floor(p * 4294967296.0);
}

/* Occupancy of configurations cfg0 .. cfg0+n_cfg-1, canonical bit layout:
 * bit s of configuration c is word c*words + s/32, bit s%32 (LSB first).
 * Counter of site s: (s/4, cfg low word, cfg high word, W<<16 | L); key = seed words;
 * site s takes output word s%4. Every output word is written by one thread (OpenMP
 * over the words of all configurations), each site with its own Philox call. */
int orc_sample(const orc_lattice *lat, double p, uint64_t seed, int64_t cfg0, int64_t n_cfg,
               uint32_t *bits) {
    if (!(p >= 0.0 && p <= 1.0) || n_cfg < 0) return ORC_EINVAL;
    int64_t n = lat->n, words = (n + 31) / 32;
    uint64_t t = orc_threshold(p);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t tag = ((uint32_t)lat->W << 16) | (uint32_t)lat->L;
    int64_t total = n_cfg * words;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t i = 0; i < total; ++i) {
        int64_t c = i / words, w = i - c * words;
        uint64_t cfg = (uint64_t)(cfg0 + c);
        uint32_t word = 0;
        for (int b = 0; b < 32; ++b) {
            int64_t s = w * 32 + b;
            if (s >= n) break;
            uint32_t ctr[4] = {(uint32_t)(s >> 2), (uint32_t)cfg, (uint32_t)(cfg >> 32), tag};
            uint32_t out[4];
            orc_philox4x32_10(ctr, key, out);
            if ((uint64_t)out[s & 3] < t) word |= 1u << b;
        }
        bits[i] = word;
    }
    return ORC_OK;
}

/* Fixed-count ensemble (Sec. II.A: Np of the N sites are chosen metallic, uniformly):
 * K = floor(N p + 1/2) sites per configuration, the K sites with the smallest 64-bit keys
 * (ties by site index). Site s takes words 2(s&1) (high) and 2(s&1)+1 (low) of the
 * Philox block with counter (s >> 1, cfg lo, cfg hi, tag | 2^31) under key = seed; the
 * top counter bit keeps these draws apart from the Bernoulli sampler's. Sorting all keys
 * is the plain definition of "the K smallest". */
typedef struct { uint64_t key; int64_t s; } orc_keyed;

static int orc_keyed_cmp(const void *a, const void *b) {
    const orc_keyed *x = (const orc_keyed *)a, *y = (const orc_keyed *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->s < y->s ? -1 : (x->s > y->s ? 1 : 0);
}

int64_t orc_fixed_count(int64_t n, double p) { return (int64_t)floor((double)n * p + 0.5); }

int orc_sample_fixed(const orc_lattice *lat, double p, uint64_t seed, int64_t cfg0, int64_t n_cfg,
                     uint32_t *bits) {
    if (!(p >= 0.0 && p <= 1.0) || n_cfg < 0) return ORC_EINVAL;
    int64_t n = lat->n, words = (n + 31) / 32, K = orc_fixed_count(n, p);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t tag = (((uint32_t)lat->W << 16) | (uint32_t)lat->L) | 0x80000000u;
    orc_keyed *ks = (orc_keyed *)malloc(sizeof(orc_keyed) * (size_t)(n > 0 ? n : 1));
    if (!ks) return ORC_ENOMEM;
    for (int64_t c = 0; c < n_cfg; ++c) {
        uint64_t cfg = (uint64_t)(cfg0 + c);
        uint32_t *b = bits + c * words;
        memset(b, 0, sizeof(uint32_t) * (size_t)words);
        for (int64_t s = 0; s < n; ++s) {
            uint32_t ctr[4] = {(uint32_t)(s >> 1), (uint32_t)cfg, (uint32_t)(cfg >> 32), tag};
            uint32_t out[4];
            orc_philox4x32_10(ctr, key, out);
            int w = 2 * (int)(s & 1);
            ks[s].key = ((uint64_t)out[w] << 32) | out[w + 1];
            ks[s].s = s;
        }
        qsort(ks, (size_t)n, sizeof(orc_keyed), orc_keyed_cmp);
        for (int64_t i = 0; i < K; ++i) b[ks[i].s >> 5] |= 1u << (ks[i].s & 31);
    }
    free(ks);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------ */
/* Markov chain: Eq. (1)-(2) with the detector j1 of Sec. II.B                     */
/* ------------------------------------------------------------------------------ */

static int bit_of(const uint32_t *b, int64_t s) { return (int)((b[s >> 5] >> (s & 31)) & 1u); }

typedef struct {
    int64_t n;      /* rows = metallic sites + 1 (detector is the last row) */
    int64_t *ptr;
    int32_t *col;
    double *val;
    int64_t *site;  /* compact row -> canonical site (-1 for the detector) */
    int64_t n_bonds_metal;
} orc_csr;

static void csr_free(orc_csr *P) {
    free(P->ptr); free(P->col); free(P->val); free(P->site);
    memset(P, 0, sizeof(*P));
}

/* Build ^(j1)P: row i of a metallic site holds 1/deg(i) for every metallic neighbour
 * and, if i is on the far surface, for the detector; deg(i) counts exactly those
 * entries so every row sums to one (Eq. 2). A metallic site with no metallic
 * neighbour keeps its mass (self-loop). The detector row is absorbing. */
static int build_P(const orc_lattice *lat, const uint32_t *bits, orc_csr *P, int64_t *map) {
    int64_t n = lat->n, m = 0;
    for (int64_t s = 0; s < n; ++s) map[s] = bit_of(bits, s) ? m++ : -1;
    P->n = m + 1;
    P->ptr = (int64_t *)malloc(sizeof(int64_t) * ((size_t)m + 2));
    P->site = (int64_t *)malloc(sizeof(int64_t) * ((size_t)m + 1));
    if (!P->ptr || !P->site) return ORC_ENOMEM;
    int64_t nnz = 0, bonds2 = 0;
    for (int64_t s = 0; s < n; ++s) {
        if (map[s] < 0) continue;
        int64_t d = 0;
        for (int64_t e = lat->nb_ptr[s]; e < lat->nb_ptr[s + 1]; ++e) d += bit_of(bits, lat->nb[e]);
        bonds2 += d;
        if (lat->is_far[s]) d += 1;
        nnz += d ? d : 1;
    }
    nnz += 1;
    P->n_bonds_metal = bonds2 / 2;
    P->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)nnz);
    P->val = (double *)malloc(sizeof(double) * (size_t)nnz);
    if (!P->col || !P->val) return ORC_ENOMEM;
    int64_t pos = 0, row = 0;
    for (int64_t s = 0; s < n; ++s) {
        if (map[s] < 0) continue;
        P->ptr[row] = pos;
        P->site[row] = s;
        int64_t d = 0;
        for (int64_t e = lat->nb_ptr[s]; e < lat->nb_ptr[s + 1]; ++e) d += bit_of(bits, lat->nb[e]);
        if (lat->is_far[s]) d += 1;
        if (d == 0) {
            P->col[pos] = (int32_t)row; P->val[pos] = 1.0; ++pos;
        } else {
            double w = 1.0 / (double)d;
            for (int64_t e = lat->nb_ptr[s]; e < lat->nb_ptr[s + 1]; ++e) {
                int64_t t = lat->nb[e];
                if (map[t] >= 0) { P->col[pos] = (int32_t)map[t]; P->val[pos] = w; ++pos; }
            }
            if (lat->is_far[s]) { P->col[pos] = (int32_t)m; P->val[pos] = w; ++pos; }
        }
        ++row;
    }
    P->ptr[m] = pos;
    P->site[m] = -1;
    P->col[pos] = (int32_t)m; P->val[pos] = 1.0; ++pos; /* absorbing detector */
    P->ptr[m + 1] = pos;
    return ORC_OK;
}

/* One Jacobi step of the forward chain: xo = xi P and the exact support
 * Ro = Ri U { j : P_ij > 0 for some i in Ri }. Returns 1 if Ro differs from Ri. */
static int markov_step(const orc_csr *P, const double *xi, double *xo, const uint8_t *Ri, uint8_t *Ro) {
    int64_t n = P->n;
    memset(xo, 0, sizeof(double) * (size_t)n);
    memcpy(Ro, Ri, (size_t)n);
    int grew = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t e = P->ptr[i]; e < P->ptr[i + 1]; ++e) {
            int32_t j = P->col[e];
            xo[j] += xi[i] * P->val[e];
            if (Ri[i] && !Ro[j]) { Ro[j] = 1; grew = 1; }
        }
    }
    return grew;
}

/* Inspection of one configuration by the Markov iteration (Sec. II.B):
 * mass 1/|S0| on each metallic start site, detector absorbing; step until the detector
 * is reached (non-zero probability in exact arithmetic, i.e. in the support), or the
 * support stops growing. N_max = min(N_b, N_occ) + 1 is kept as an assertion. */
static int inspect_markov_one(const orc_lattice *lat, const uint32_t *bits, uint8_t *perc,
                              int32_t *steps, double *hitmass) {
    int64_t n = lat->n;
    int64_t *map = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    if (!map) return ORC_ENOMEM;
    orc_csr P; memset(&P, 0, sizeof(P));
    int rc = build_P(lat, bits, &P, map);
    if (rc) { free(map); csr_free(&P); return rc; }
    int64_t m = P.n - 1; /* metallic sites; detector = m */
    double *x = (double *)calloc((size_t)P.n, sizeof(double));
    double *y = (double *)calloc((size_t)P.n, sizeof(double));
    uint8_t *R = (uint8_t *)calloc((size_t)P.n, 1);
    uint8_t *R2 = (uint8_t *)calloc((size_t)P.n, 1);
    if (!x || !y || !R || !R2) { rc = ORC_ENOMEM; goto done; }
    int64_t s0 = 0;
    for (int64_t i = 0; i < m; ++i) if (lat->is_start[P.site[i]]) ++s0;
    *perc = 0; *steps = 0; *hitmass = 0.0;
    if (s0 == 0) goto done;
    for (int64_t i = 0; i < m; ++i)
        if (lat->is_start[P.site[i]]) { x[i] = 1.0 / (double)s0; R[i] = 1; }
    int64_t nmax = (P.n_bonds_metal < m ? P.n_bonds_metal : m) + 1;
    for (int64_t it = 1;; ++it) {
        int grew = markov_step(&P, x, y, R, R2);
        double *tx = x; x = y; y = tx;
        uint8_t *tR = R; R = R2; R2 = tR;
        if (R[m]) { *perc = 1; *steps = (int32_t)it; *hitmass = x[m]; break; }
        if (!grew) { *perc = 0; *steps = (int32_t)it; break; }
        if (it >= nmax) { rc = ORC_ECAP; break; }
    }
done:
    free(x); free(y); free(R); free(R2); free(map); csr_free(&P);
    return rc;
}

int orc_inspect_markov(const orc_lattice *lat, const uint32_t *bits, int64_t n_cfg, uint8_t *perc,
                       int32_t *steps, double *hitmass, int nthreads) {
    int64_t words = (lat->n + 31) / 32;
    int err = 0;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(| : err)
#endif
    for (int64_t c = 0; c < n_cfg; ++c) {
        double hm = 0.0;
        int rc = inspect_markov_one(lat, bits + c * words, perc + c, steps + c, &hm);
        if (hitmass) hitmass[c] = hm;
        if (rc) err |= 1;
    }
    (void)nthreads;
    return err ? ORC_ECAP : ORC_OK;
}

/* Exactly K forward steps without early exit. x has n+1 entries (canonical site order,
 * zero at insulating sites, detector last); reach likewise (0/1). */
int orc_state_after(const orc_lattice *lat, const uint32_t *bits, int32_t K, double *x_out,
                    uint8_t *reach_out) {
    if (K < 0) return ORC_EINVAL;
    int64_t n = lat->n;
    int64_t *map = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    if (!map) return ORC_ENOMEM;
    orc_csr P; memset(&P, 0, sizeof(P));
    int rc = build_P(lat, bits, &P, map);
    if (rc) { free(map); csr_free(&P); return rc; }
    int64_t m = P.n - 1;
    double *x = (double *)calloc((size_t)P.n, sizeof(double));
    double *y = (double *)calloc((size_t)P.n, sizeof(double));
    uint8_t *R = (uint8_t *)calloc((size_t)P.n, 1);
    uint8_t *R2 = (uint8_t *)calloc((size_t)P.n, 1);
    if (!x || !y || !R || !R2) { rc = ORC_ENOMEM; goto done; }
    int64_t s0 = 0;
    for (int64_t i = 0; i < m; ++i) if (lat->is_start[P.site[i]]) ++s0;
    if (s0 > 0)
        for (int64_t i = 0; i < m; ++i)
            if (lat->is_start[P.site[i]]) { x[i] = 1.0 / (double)s0; R[i] = 1; }
    for (int32_t it = 0; it < K; ++it) {
        markov_step(&P, x, y, R, R2);
        double *tx = x; x = y; y = tx;
        uint8_t *tR = R; R = R2; R2 = tR;
    }
    for (int64_t s = 0; s <= n; ++s) { x_out[s] = 0.0; reach_out[s] = 0; }
    for (int64_t i = 0; i < m; ++i) { x_out[P.site[i]] = x[i]; reach_out[P.site[i]] = R[i]; }
    x_out[n] = x[m]; reach_out[n] = R[m];
done:
    free(x); free(y); free(R); free(R2); free(map); csr_free(&P);
    return rc;
}

/* Row sums of ^(j1)P for a configuration (pin: every row sums to one, Sec. II.B). */
int orc_row_sums(const orc_lattice *lat, const uint32_t *bits, double *sums, int64_t *n_rows) {
    int64_t n = lat->n;
    int64_t *map = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    if (!map) return ORC_ENOMEM;
    orc_csr P; memset(&P, 0, sizeof(P));
    int rc = build_P(lat, bits, &P, map);
    if (!rc) {
        *n_rows = P.n;
        for (int64_t i = 0; i < P.n; ++i) {
            double s = 0.0;
            for (int64_t e = P.ptr[i]; e < P.ptr[i + 1]; ++e) s += P.val[e];
            sums[i] = s;
        }
    }
    free(map); csr_free(&P);
    return rc;
}

/* ------------------------------------------------------------------------------ */
/* Eq. (3)-(4) on an arbitrary row-stochastic matrix, and its forward counterpart  */
/* ------------------------------------------------------------------------------ */

/* f^(1) = column j0 of P; f^(m) = ^(j0)P f^(m-1), where ^(j0)P is P with column j0
 * set to zero. f[(m-1)*n + i] = P_i[first hit of j0 at step m], m = 1..M. */
int orc_eq3_backward(int64_t n, const int64_t *ptr, const int32_t *col, const double *val, int32_t j0,
                     int32_t M, double *f) {
    if (n <= 0 || j0 < 0 || j0 >= n || M < 1) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        double v = 0.0;
        for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) if (col[e] == j0) v += val[e];
        f[i] = v;
    }
    for (int32_t m = 2; m <= M; ++m) {
        const double *prev = f + (int64_t)(m - 2) * n;
        double *cur = f + (int64_t)(m - 1) * n;
        for (int64_t i = 0; i < n; ++i) {
            double v = 0.0;
            for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) if (col[e] != j0) v += val[e] * prev[col[e]];
            cur[i] = v;
        }
    }
    return ORC_OK;
}

/* Eq. 3 for every source at once on the fiber: out[s] = P_s[the walk from tube s first
 * reaches the detector j1 at step M] = [(^(j1)P)^(M-1) f](s), f = the j1 column of P (the
 * detector's entry of each row), ^(j1)P = P with that column zeroed; 0 for insulating
 * tubes. The plain backward recursion over the explicit CSR, in FP64. */
int orc_first_passage_all(const orc_lattice *lat, const uint32_t *bits, int32_t M, double *out) {
    if (M < 1) return ORC_EINVAL;
    int64_t n = lat->n;
    int64_t *map = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    if (!map) return ORC_ENOMEM;
    orc_csr P; memset(&P, 0, sizeof(P));
    int rc = build_P(lat, bits, &P, map);
    if (rc) { free(map); csr_free(&P); return rc; }
    int64_t m = P.n - 1, j1 = m;
    double *f = (double *)calloc((size_t)P.n, sizeof(double));
    double *g = (double *)calloc((size_t)P.n, sizeof(double));
    if (!f || !g) { rc = ORC_ENOMEM; goto done; }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t e = P.ptr[i]; e < P.ptr[i + 1]; ++e) if (P.col[e] == j1) f[i] += P.val[e];
    for (int32_t it = 1; it < M; ++it) {
        for (int64_t i = 0; i < m; ++i) {
            double v = 0.0;
            for (int64_t e = P.ptr[i]; e < P.ptr[i + 1]; ++e) if (P.col[e] != j1) v += P.val[e] * f[P.col[e]];
            g[i] = v;
        }
        double *t = f; f = g; g = t;
    }
    for (int64_t s = 0; s < n; ++s) out[s] = 0.0;
    for (int64_t i = 0; i < m; ++i) out[P.site[i]] = f[i];
done:
    free(f); free(g); free(map); csr_free(&P);
    return rc;
}

/* Forward form: x^(0) = x0, the row of j0 replaced by an absorbing self-loop, x <- x P.
 * hit[m-1] = x^(m)_j0 - x^(m-1)_j0 = P_x0[first hit of j0 at step m]. */
int orc_first_passage_forward(int64_t n, const int64_t *ptr, const int32_t *col, const double *val,
                              int32_t j0, const double *x0, int32_t M, double *hit) {
    if (n <= 0 || j0 < 0 || j0 >= n || M < 1) return ORC_EINVAL;
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    if (!x || !y) { free(x); free(y); return ORC_ENOMEM; }
    memcpy(x, x0, sizeof(double) * (size_t)n);
    double absorbed = x[j0];
    for (int32_t m = 1; m <= M; ++m) {
        memset(y, 0, sizeof(double) * (size_t)n);
        for (int64_t i = 0; i < n; ++i) {
            if (i == j0) { y[j0] += x[j0]; continue; }
            for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) y[col[e]] += x[i] * val[e];
        }
        hit[m - 1] = y[j0] - absorbed;
        absorbed = y[j0];
        double *t = x; x = y; y = t;
    }
    free(x); free(y);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------ */
/* Plain definition: breadth-first search and union-find                           */
/* ------------------------------------------------------------------------------ */

/* Multi-source BFS from the metallic start sites over metallic neighbours.
 * perc = some metallic far site is reached; steps = the iteration count the Markov
 * inspection must take: (distance to the nearest reached far site) + 1 if percolating,
 * else (largest distance reached) + 1, and 0 when no start site is metallic. */
static int bfs_one(const orc_lattice *lat, const uint32_t *bits, uint8_t *perc, int32_t *steps,
                   int32_t *dist_out) {
    int64_t n = lat->n;
    int32_t *dist = dist_out ? dist_out : (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    if (!dist || !queue) { if (!dist_out) free(dist); free(queue); return ORC_ENOMEM; }
    int64_t head = 0, tail = 0;
    for (int64_t s = 0; s < n; ++s) {
        dist[s] = -1;
        if (lat->is_start[s] && bit_of(bits, s)) { dist[s] = 0; queue[tail++] = s; }
    }
    *perc = 0; *steps = 0;
    if (tail > 0) {
        int32_t far_d = -1, max_d = 0;
        while (head < tail) {
            int64_t s = queue[head++];
            if (dist[s] > max_d) max_d = dist[s];
            if (lat->is_far[s] && (far_d < 0 || dist[s] < far_d)) far_d = dist[s];
            for (int64_t e = lat->nb_ptr[s]; e < lat->nb_ptr[s + 1]; ++e) {
                int64_t t = lat->nb[e];
                if (dist[t] < 0 && bit_of(bits, t)) { dist[t] = dist[s] + 1; queue[tail++] = t; }
            }
        }
        if (far_d >= 0) { *perc = 1; *steps = far_d + 1; }
        else { *perc = 0; *steps = max_d + 1; }
    }
    if (!dist_out) free(dist);
    free(queue);
    return ORC_OK;
}

int orc_inspect_bfs(const orc_lattice *lat, const uint32_t *bits, int64_t n_cfg, uint8_t *perc,
                    int32_t *steps, int nthreads) {
    int64_t words = (lat->n + 31) / 32;
    int err = 0;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads) reduction(| : err)
#endif
    for (int64_t c = 0; c < n_cfg; ++c)
        if (bfs_one(lat, bits + c * words, perc + c, steps + c, NULL)) err |= 1;
    (void)nthreads;
    return err ? ORC_ENOMEM : ORC_OK;
}

/* Distances from the metallic start set (-1 where unreached), for one configuration. */
int orc_bfs_dist(const orc_lattice *lat, const uint32_t *bits, int32_t *dist) {
    uint8_t p; int32_t s;
    return bfs_one(lat, bits, &p, &s, dist);
}

static int64_t uf_find(int64_t *parent, int64_t a) {
    while (parent[a] != a) { parent[a] = parent[parent[a]]; a = parent[a]; }
    return a;
}

int orc_inspect_uf(const orc_lattice *lat, const uint32_t *bits, int64_t n_cfg, uint8_t *perc) {
    int64_t n = lat->n, words = (n + 31) / 32;
    /* two virtual nodes: n = start side, n+1 = far side */
    int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 2));
    if (!parent) return ORC_ENOMEM;
    for (int64_t c = 0; c < n_cfg; ++c) {
        const uint32_t *b = bits + c * words;
        for (int64_t i = 0; i < n + 2; ++i) parent[i] = i;
        for (int64_t s = 0; s < n; ++s) {
            if (!bit_of(b, s)) continue;
            if (lat->is_start[s]) { int64_t a = uf_find(parent, s), z = uf_find(parent, n); if (a != z) parent[a] = z; }
            if (lat->is_far[s]) { int64_t a = uf_find(parent, s), z = uf_find(parent, n + 1); if (a != z) parent[a] = z; }
            for (int64_t e = lat->nb_ptr[s]; e < lat->nb_ptr[s + 1]; ++e) {
                int64_t t = lat->nb[e];
                if (t < s || !bit_of(b, t)) continue;
                int64_t a = uf_find(parent, s), z = uf_find(parent, t);
                if (a != z) parent[a] = z;
            }
        }
        perc[c] = uf_find(parent, n) == uf_find(parent, n + 1);
    }
    free(parent);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------ */
/* Exhaustive enumeration of all 2^N configurations (N <= 24)                      */
/* ------------------------------------------------------------------------------ */

/* a[k] = number of percolating configurations with exactly k metallic sites, by BFS
 * (method = 0) or by the Markov iteration (method = 1). */
int orc_exhaustive(const orc_lattice *lat, int method, int64_t *a) {
    int64_t n = lat->n;
    if (n > 24) return ORC_EINVAL;
    for (int64_t k = 0; k <= n; ++k) a[k] = 0;
    uint64_t total = (uint64_t)1 << n;
    int err = 0;
#ifdef _OPENMP
#pragma omp parallel
#endif
    {
        int64_t local[25] = {0};
        int lerr = 0;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t mask = 0; mask < (int64_t)total; ++mask) {
            uint32_t b[1] = {(uint32_t)mask};
            uint8_t p = 0; int32_t st = 0; double hm = 0.0;
            int rc = method ? inspect_markov_one(lat, b, &p, &st, &hm) : bfs_one(lat, b, &p, &st, NULL);
            if (rc) lerr = 1;
            if (p) local[__builtin_popcountll((unsigned long long)mask)]++;
        }
#ifdef _OPENMP
#pragma omp critical
#endif
        {
            for (int64_t k = 0; k <= n; ++k) a[k] += local[k];
            err |= lerr;
        }
    }
    return err ? ORC_ECAP : ORC_OK;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
