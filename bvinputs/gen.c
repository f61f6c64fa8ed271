/*
 * Seeded synthetic inputs for the compressed-graph product: graph generators
 * and the encoder of the project's Boldi-Vigna-style bitstream.
 *
 * This file is input production only.  It computes no product, no PageRank
 * and decodes nothing; both the CPU oracle and the HIP library consume what
 * it writes (the adjacency lists as CSR, and the bitstream), each with a
 * decoder of its own.
 *
 * Graph models (synthetic stand-ins for the web and social crawls the paper
 * measures on, Section "Experimental Evaluation", Table 1):
 *   - web-like copying model: node i picks a prototype among the previous
 *     `pw` nodes, copies each of its links with probability p_copy, then adds
 *     links starting near i at geometric gaps, half of them as runs of >= 4
 *     consecutive ids (the copy property and locality the paper's Section
 *     "Our Approach" relies on);
 *   - social-like model: out-degree from a truncated shifted power law, weak
 *     copying, uniform random remaining targets, optional BFS renumbering.
 *
 * Bitstream (project-defined; the paper only names list referencing within a
 * window W, copy/skip marking, differential compression and codes for natural
 * numbers, Section "Our Approach").  Little-endian 64-byte header:
 *   0 "BVMV" | 4 u32 version=1 | 8 u64 n | 16 u64 m | 24 u32 W | 28 u32 R
 *   32 u32 Lmin | 36 u32 zeta_k | 40 u32 stride S | 44 u32 0 | 48 u64 body_bits
 *   56 u64 nseg ; then nseg u64 bit offsets (offset of node k*S);
 *   then the body, MSB-first bit order, zero padded to a multiple of 8 bytes.
 * Per node i (codes: unary(x)= x zeros then a one; gamma(x) on x+1; zeta_k(x)
 * on x+1; nu(z)= 2z for z>=0, 2|z|-1 for z<0):
 *   gamma(d_i); if d_i==0 done.
 *   if W>0: unary(g), g = i - r_i in [0,W], 0 = no reference.  With a segment
 *     table (S > 0) a reference never crosses a multiple of S, so each
 *     segment of S nodes decodes on its own.
 *   if g>0: gamma(b) explicit blocks over the reference's list; block 0 (copy)
 *     gamma(len), later blocks gamma(len-1), alternating copy/skip; the rest of
 *     the reference list is copied if b is even, skipped if b is odd.
 *   E = list minus copied entries, |E| = d_i - |copied|.
 *   if |E| >= Lmin: gamma(#intervals); interval k: start gamma(nu(s-i)) for
 *     k=0 else gamma(s - prev_last - 2); length gamma(len - Lmin).  Intervals
 *     are the maximal runs of consecutive ids of E of length >= Lmin.
 *   residuals (rest of E, ascending): first zeta_k(nu(j-i)), then
 *     zeta_k(j - prev - 1).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ rng */
typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64(uint64_t *x) {
  uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static void rng_seed(rng_t *r, uint64_t seed) {
  uint64_t x = seed;
  for (int k = 0; k < 4; ++k) r->s[k] = splitmix64(&x);
}
static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
/* xoshiro256** (Blackman & Vigna) */
static inline uint64_t rng_next(rng_t *r) {
  uint64_t *s = r->s;
  const uint64_t res = rotl64(s[1] * 5, 7) * 9;
  const uint64_t t = s[1] << 17;
  s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
  s[2] ^= t; s[3] = rotl64(s[3], 45);
  return res;
}
static inline double rng_u01(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }
static inline double rng_u01_open(rng_t *r) { return ((double)(rng_next(r) >> 11) + 1.0) * 0x1.0p-53; }
/* uniform integer in [0, span) */
static inline uint64_t rng_below(rng_t *r, uint64_t span) {
  return (uint64_t)(((unsigned __int128)rng_next(r) * span) >> 64);
}
/* geometric on {1,2,...} with the given mean (>= 1) */
static inline int64_t rng_geom(rng_t *r, double mean) {
  if (mean <= 1.0) return 1;
  const double p = 1.0 / mean;
  return 1 + (int64_t)floor(log(rng_u01_open(r)) / log1p(-p));
}
/* Poisson by Knuth's product method, split into pieces of mean <= 20 */
static int64_t rng_poisson(rng_t *r, double lam) {
  int64_t total = 0;
  while (lam > 0) {
    const double piece = lam > 20.0 ? 20.0 : lam;
    lam -= piece;
    const double L = exp(-piece);
    double p = 1.0;
    int64_t k = -1;
    do { ++k; p *= rng_u01_open(r); } while (p > L);
    total += k;
  }
  return total;
}

/* ------------------------------------------------------------ helpers */
static void sort_u32(uint32_t *a, int64_t n) {
  /* iterative quicksort with insertion sort for short ranges */
  int64_t stack[128];
  int sp = 0;
  stack[sp++] = 0; stack[sp++] = n - 1;
  while (sp) {
    int64_t hi = stack[--sp], lo = stack[--sp];
    while (hi - lo > 24) {
      int64_t mid = lo + (hi - lo) / 2;
      uint32_t a0 = a[lo], a1 = a[mid], a2 = a[hi];
      uint32_t piv = a0 < a1 ? (a1 < a2 ? a1 : (a0 < a2 ? a2 : a0)) : (a0 < a2 ? a0 : (a1 < a2 ? a2 : a1));
      int64_t i = lo, j = hi;
      while (i <= j) {
        while (a[i] < piv) ++i;
        while (a[j] > piv) --j;
        if (i <= j) { uint32_t t = a[i]; a[i] = a[j]; a[j] = t; ++i; --j; }
      }
      if (j - lo < hi - i) { if (i < hi) { stack[sp++] = i; stack[sp++] = hi; } hi = j; }
      else { if (lo < j) { stack[sp++] = lo; stack[sp++] = j; } lo = i; }
    }
    for (int64_t i = lo + 1; i <= hi; ++i) {
      uint32_t v = a[i]; int64_t j = i - 1;
      while (j >= lo && a[j] > v) { a[j + 1] = a[j]; --j; }
      a[j + 1] = v;
    }
  }
}

typedef struct { uint32_t *col; size_t len, cap; } colbuf_t;
static int colbuf_reserve(colbuf_t *b, size_t extra) {
  if (b->len + extra <= b->cap) return 0;
  size_t nc = b->cap ? b->cap : 1024;
  while (nc < b->len + extra) nc += nc / 2 + 1024;
  uint32_t *p = (uint32_t *)realloc(b->col, nc * sizeof(uint32_t));
  if (!p) return -1;
  b->col = p; b->cap = nc;
  return 0;
}

void bvi_free(void *p) { free(p); }

/* ------------------------------------------------------ web-like model */
int bvi_web_graph(int64_t n, double mean_deg, uint64_t seed, int pw, double p_copy,
                  double gap_mean, uint64_t **rowptr_out, uint32_t **col_out, int64_t *m_out) {
  if (n <= 0 || n >= (int64_t)0xFFFFFFFFll || mean_deg < 1.0 || pw < 0) return -1;
  rng_t r; rng_seed(&r, seed);
  uint64_t *rowptr = (uint64_t *)malloc((size_t)(n + 1) * sizeof(uint64_t));
  uint32_t *mark = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
  size_t rcap = 4096;
  uint32_t *row = (uint32_t *)malloc(rcap * sizeof(uint32_t));
  colbuf_t cb = {0, 0, 0};
  if (!rowptr || !mark || !row || colbuf_reserve(&cb, (size_t)((double)n * (mean_deg + 1.0) * 1.05) + 64)) {
    free(rowptr); free(mark); free(row); free(cb.col); return -2;
  }
  rowptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    const uint32_t stamp = (uint32_t)(i + 1);
    int64_t cnt = 0;
    int64_t D = 1 + rng_poisson(&r, mean_deg - 1.0);
    if (D > n - 1) D = n - 1;
    int64_t need_cap = D + 8;
    if (i > 0) {
      int64_t lo = i - pw; if (lo < 0) lo = 0;
      int64_t q = lo + (int64_t)rng_below(&r, (uint64_t)(i - lo));
      need_cap += (int64_t)(rowptr[q + 1] - rowptr[q]);
      if ((size_t)need_cap > rcap) { rcap = (size_t)need_cap * 2; row = (uint32_t *)realloc(row, rcap * sizeof(uint32_t)); }
      for (uint64_t k = rowptr[q]; k < rowptr[q + 1]; ++k) {
        uint32_t t = cb.col[k];
        if (rng_u01(&r) < p_copy && (int64_t)t != i && mark[t] != stamp) { mark[t] = stamp; row[cnt++] = t; }
      }
    } else if ((size_t)need_cap > rcap) {
      rcap = (size_t)need_cap * 2; row = (uint32_t *)realloc(row, rcap * sizeof(uint32_t));
    }
    int64_t need = D - cnt;
    if (need > 0) {
      int64_t cur = i - 12 + rng_geom(&r, gap_mean);
      int64_t guard = 0;
      while (need > 0 && guard < 64 + 16 * D) {
        int64_t L = (rng_u01(&r) < 0.5) ? 3 + rng_geom(&r, 2.0) : 1;
        for (int64_t t = 0; t < L && need > 0; ++t) {
          int64_t id = (cur + t) % n; if (id < 0) id += n;
          if (id != i && mark[id] != stamp) { mark[id] = stamp; row[cnt++] = (uint32_t)id; --need; }
        }
        cur += L - 1 + rng_geom(&r, gap_mean);
        ++guard;
      }
    }
    sort_u32(row, cnt);
    if (colbuf_reserve(&cb, (size_t)cnt)) { free(rowptr); free(mark); free(row); free(cb.col); return -2; }
    memcpy(cb.col + cb.len, row, (size_t)cnt * sizeof(uint32_t));
    cb.len += (size_t)cnt;
    rowptr[i + 1] = cb.len;
  }
  free(mark); free(row);
  *rowptr_out = rowptr; *col_out = cb.col; *m_out = (int64_t)cb.len;
  return 0;
}

/* --------------------------------------------------- social-like model */
/* mean of P(k) ~ (k+s)^-e on k in [1,kmax] */
static double plaw_mean(double s, double e, int64_t kmax) {
  double num = 0, den = 0;
  for (int64_t k = 1; k <= kmax; ++k) { double w = pow((double)k + s, -e); num += w * (double)k; den += w; }
  return num / den;
}

double bvi_powerlaw_shift(double mean_deg, int64_t kmax, double expo) {
  double lo = 0.0, hi = 1.0;
  if (plaw_mean(0.0, expo, kmax) >= mean_deg) return 0.0;
  while (plaw_mean(hi, expo, kmax) < mean_deg && hi < 1e7) hi *= 2;
  for (int it = 0; it < 100; ++it) {
    double mid = 0.5 * (lo + hi);
    if (plaw_mean(mid, expo, kmax) < mean_deg) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

int bvi_social_graph(int64_t n, double mean_deg, int64_t kmax, double expo, uint64_t seed, int pw,
                     double p_copy, int bfs, uint64_t **rowptr_out, uint32_t **col_out, int64_t *m_out) {
  if (n <= 1 || n >= (int64_t)0xFFFFFFFFll || kmax < 1 || mean_deg < 1.0) return -1;
  if (kmax > n - 1) kmax = n - 1;
  const double s = bvi_powerlaw_shift(mean_deg, kmax, expo);
  double *cdf = (double *)malloc((size_t)kmax * sizeof(double));
  double acc = 0;
  for (int64_t k = 1; k <= kmax; ++k) { acc += pow((double)k + s, -expo); cdf[k - 1] = acc; }
  for (int64_t k = 0; k < kmax; ++k) cdf[k] /= acc;
  rng_t r; rng_seed(&r, seed);
  uint64_t *rowptr = (uint64_t *)malloc((size_t)(n + 1) * sizeof(uint64_t));
  uint32_t *mark = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
  size_t rcap = (size_t)kmax + 64;
  uint32_t *row = (uint32_t *)malloc(rcap * sizeof(uint32_t));
  colbuf_t cb = {0, 0, 0};
  if (!cdf || !rowptr || !mark || !row || colbuf_reserve(&cb, (size_t)((double)n * mean_deg * 1.05) + 64)) {
    free(cdf); free(rowptr); free(mark); free(row); free(cb.col); return -2;
  }
  rowptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    const uint32_t stamp = (uint32_t)(i + 1);
    double u = rng_u01(&r);
    int64_t lo = 0, hi = kmax - 1;
    while (lo < hi) { int64_t mid = (lo + hi) / 2; if (cdf[mid] < u) lo = mid + 1; else hi = mid; }
    int64_t D = lo + 1, cnt = 0;
    if (i > 0) {
      int64_t plo = i - pw; if (plo < 0) plo = 0;
      int64_t q = plo + (int64_t)rng_below(&r, (uint64_t)(i - plo));
      for (uint64_t k = rowptr[q]; k < rowptr[q + 1] && cnt < D; ++k) {
        uint32_t t = cb.col[k];
        if (rng_u01(&r) < p_copy && (int64_t)t != i && mark[t] != stamp) { mark[t] = stamp; row[cnt++] = t; }
      }
    }
    while (cnt < D) {
      uint32_t t = (uint32_t)rng_below(&r, (uint64_t)n);
      if ((int64_t)t != i && mark[t] != stamp) { mark[t] = stamp; row[cnt++] = t; }
    }
    sort_u32(row, cnt);
    if (colbuf_reserve(&cb, (size_t)cnt)) { free(cdf); free(rowptr); free(mark); free(row); free(cb.col); return -2; }
    memcpy(cb.col + cb.len, row, (size_t)cnt * sizeof(uint32_t));
    cb.len += (size_t)cnt;
    rowptr[i + 1] = cb.len;
  }
  free(cdf); free(row);
  if (bfs) {
    /* BFS over out-links from node 0, neighbours in ascending id order,
       restarting from the smallest unvisited id; new id = visit order. */
    uint32_t *newid = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    uint32_t *queue = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    memset(newid, 0xFF, (size_t)n * sizeof(uint32_t));
    int64_t head = 0, tail = 0;
    for (int64_t st = 0; st < n; ++st) {
      if (newid[st] != 0xFFFFFFFFu) continue;
      newid[st] = (uint32_t)tail; queue[tail++] = (uint32_t)st;
      while (head < tail) {
        uint32_t u = queue[head++];
        for (uint64_t k = rowptr[u]; k < rowptr[u + 1]; ++k) {
          uint32_t v = cb.col[k];
          if (newid[v] == 0xFFFFFFFFu) { newid[v] = (uint32_t)tail; queue[tail++] = v; }
        }
      }
    }
    /* queue[k] = old id of new node k */
    uint64_t *nrp = (uint64_t *)malloc((size_t)(n + 1) * sizeof(uint64_t));
    uint32_t *ncol = (uint32_t *)malloc(cb.len * sizeof(uint32_t) + 4);
    nrp[0] = 0;
    for (int64_t k = 0; k < n; ++k) {
      uint32_t u = queue[k];
      uint64_t d = rowptr[u + 1] - rowptr[u];
      uint32_t *dst = ncol + nrp[k];
      for (uint64_t t = 0; t < d; ++t) dst[t] = newid[cb.col[rowptr[u] + t]];
      sort_u32(dst, (int64_t)d);
      nrp[k + 1] = nrp[k] + d;
    }
    free(newid); free(queue); free(rowptr); free(cb.col);
    rowptr = nrp; cb.col = ncol;
  }
  free(mark);
  *rowptr_out = rowptr; *col_out = cb.col; *m_out = (int64_t)rowptr[n];
  return 0;
}

/* ------------------------------------------------------------ encoder */
static inline int floor_log2_u64(uint64_t v) { return 63 - __builtin_clzll(v); }
static inline int ceil_log2_u64(uint64_t v) { return v <= 1 ? 0 : 64 - __builtin_clzll(v - 1); }
static inline uint64_t nu_map(int64_t z) { return z >= 0 ? (uint64_t)(2 * z) : (uint64_t)(2 * (-z) - 1); }

typedef struct { uint64_t *w; size_t capw; uint64_t nbits; int fail; } bitw_t;

static void bw_put(bitw_t *b, uint64_t val, int nb) { /* low nb bits of val, MSB first, nb <= 64 */
  if (nb == 0) return;
  if (nb < 64) val &= ((1ull << nb) - 1);
  size_t need = (size_t)((b->nbits + (uint64_t)nb + 63) / 64) + 1;
  if (need > b->capw) {
    size_t nc = b->capw ? b->capw * 2 : 1024;
    while (nc < need) nc *= 2;
    uint64_t *p = (uint64_t *)realloc(b->w, nc * sizeof(uint64_t));
    if (!p) { b->fail = 1; return; }
    memset(p + b->capw, 0, (nc - b->capw) * sizeof(uint64_t));
    b->w = p; b->capw = nc;
  }
  size_t wi = (size_t)(b->nbits >> 6);
  int used = (int)(b->nbits & 63), room = 64 - used;
  if (nb <= room) {
    b->w[wi] |= val << (room - nb);
  } else {
    b->w[wi] |= val >> (nb - room);
    b->w[wi + 1] |= val << (64 - (nb - room));
  }
  b->nbits += (uint64_t)nb;
}
static void bw_unary(bitw_t *b, uint64_t x) {
  while (x >= 63) { bw_put(b, 0, 63); x -= 63; }
  bw_put(b, 1, (int)x + 1);
}
static void bw_gamma(bitw_t *b, uint64_t x) {
  uint64_t v = x + 1; int nb = floor_log2_u64(v);
  bw_unary(b, (uint64_t)nb); bw_put(b, v, nb);
}
static void bw_zeta(bitw_t *b, uint64_t x, int k) {
  uint64_t v = x + 1; int h = floor_log2_u64(v) / k;
  bw_unary(b, (uint64_t)h);
  uint64_t left = 1ull << (h * k), zmax = (1ull << ((h + 1) * k)) - left, z = v - left;
  int sb = ceil_log2_u64(zmax);
  uint64_t thr = (1ull << sb) - zmax;
  if (z < thr) bw_put(b, z, sb - 1); else bw_put(b, z + thr, sb);
}
static inline uint64_t len_gamma(uint64_t x) { return 2 * (uint64_t)floor_log2_u64(x + 1) + 1; }
static inline uint64_t len_zeta(uint64_t x, int k) {
  uint64_t v = x + 1; int h = floor_log2_u64(v) / k;
  uint64_t left = 1ull << (h * k), zmax = (1ull << ((h + 1) * k)) - left, z = v - left;
  int sb = ceil_log2_u64(zmax);
  uint64_t thr = (1ull << sb) - zmax;
  return (uint64_t)h + 1 + (uint64_t)(z < thr ? sb - 1 : sb);
}

typedef struct { int W, R, Lmin, zk; } encp_t;

/* Encode (bw != NULL) or just cost in bits (bw == NULL) row i against the
   reference list Lr (g > 0) or none (g == 0).  scratch must hold d_i entries. */
static uint64_t row_code(bitw_t *bw, const encp_t *P, int64_t i, const uint32_t *Li, int64_t di,
                         const uint32_t *Lr, int64_t dr, int g, uint32_t *scratch) {
  uint64_t bits = len_gamma((uint64_t)di);
  if (bw) bw_gamma(bw, (uint64_t)di);
  if (di == 0) return bits;
  if (P->W > 0) { bits += (uint64_t)g + 1; if (bw) bw_unary(bw, (uint64_t)g); }
  const uint32_t *E = Li; int64_t ne = di;
  if (g > 0) {
    /* copy/skip blocks over Lr: blocks [c0, s1, c2, ...]; explicit b = B-1 */
    int64_t a = 0, nblk = 0, cur_len = 0; int cur_copy = 1;
    /* first pass: count blocks and their cost */
    uint64_t blk_bits = 0;
    int64_t ib = 0;
    /* extras written to scratch */
    ne = 0;
    for (int64_t k = 0; k < dr; ++k) {
      const uint32_t v = Lr[k];
      while (ib < di && Li[ib] < v) scratch[ne++] = Li[ib++];
      int copied = (ib < di && Li[ib] == v);
      if (copied) ++ib;
      if (copied == cur_copy) ++cur_len;
      else {
        blk_bits += nblk == 0 ? len_gamma((uint64_t)cur_len) : len_gamma((uint64_t)cur_len - 1);
        ++nblk; cur_copy = copied; cur_len = 1;
      }
    }
    while (ib < di) scratch[ne++] = Li[ib++];
    /* the final block (cur) is implicit */
    bits += len_gamma((uint64_t)nblk) + blk_bits;
    if (bw) {
      bw_gamma(bw, (uint64_t)nblk);
      int64_t written = 0; cur_copy = 1; cur_len = 0; ib = 0;
      for (int64_t k = 0; k < dr && written < nblk; ++k) {
        const uint32_t v = Lr[k];
        while (ib < di && Li[ib] < v) ++ib;
        int copied = (ib < di && Li[ib] == v);
        if (copied) ++ib;
        if (copied == cur_copy) ++cur_len;
        else {
          if (written == 0) bw_gamma(bw, (uint64_t)cur_len); else bw_gamma(bw, (uint64_t)cur_len - 1);
          ++written; cur_copy = copied; cur_len = 1;
        }
      }
    }
    (void)a;
    E = scratch;
  }
  if (ne == 0) return bits;
  /* intervals: maximal runs of E of length >= Lmin */
  const int Lmin = P->Lmin;
  int64_t nint = 0;
  if (ne >= Lmin) {
    for (int64_t k = 0; k < ne;) {
      int64_t e = k + 1;
      while (e < ne && E[e] == E[e - 1] + 1) ++e;
      if (e - k >= Lmin) ++nint;
      k = e;
    }
    bits += len_gamma((uint64_t)nint);
    if (bw) bw_gamma(bw, (uint64_t)nint);
  }
  int64_t prev_last = -1, idx = 0;
  if (nint > 0) {
    for (int64_t k = 0; k < ne;) {
      int64_t e = k + 1;
      while (e < ne && E[e] == E[e - 1] + 1) ++e;
      if (e - k >= Lmin) {
        uint64_t sc = idx == 0 ? nu_map((int64_t)E[k] - i) : (uint64_t)((int64_t)E[k] - prev_last - 2);
        uint64_t lc = (uint64_t)(e - k - Lmin);
        bits += len_gamma(sc) + len_gamma(lc);
        if (bw) { bw_gamma(bw, sc); bw_gamma(bw, lc); }
        prev_last = (int64_t)E[e - 1]; ++idx;
      }
      k = e;
    }
  }
  /* residuals */
  int64_t prev = -1; int first = 1;
  for (int64_t k = 0; k < ne;) {
    int64_t e = k + 1;
    while (e < ne && E[e] == E[e - 1] + 1) ++e;
    if (nint > 0 && e - k >= Lmin) { k = e; continue; }
    for (int64_t t = k; t < e; ++t) {
      uint64_t c = first ? nu_map((int64_t)E[t] - i) : (uint64_t)((int64_t)E[t] - prev - 1);
      bits += len_zeta(c, P->zk);
      if (bw) bw_zeta(bw, c, P->zk);
      prev = (int64_t)E[t]; first = 0;
    }
    k = e;
  }
  return bits;
}

typedef struct {
  const encp_t *P; int64_t n; const uint64_t *rp; const uint32_t *col;
  int64_t lo, hi; uint64_t *cost; /* cost[(i)*(W+1)+g], UINT64_MAX if invalid */
  const uint8_t *gsel; bitw_t bw; int phase; int64_t stride;
} enc_job_t;

static void *enc_worker(void *arg) {
  enc_job_t *J = (enc_job_t *)arg;
  const encp_t *P = J->P;
  int64_t maxd = 0;
  for (int64_t i = J->lo; i < J->hi; ++i) { int64_t d = (int64_t)(J->rp[i + 1] - J->rp[i]); if (d > maxd) maxd = d; }
  uint32_t *scratch = (uint32_t *)malloc((size_t)(maxd + 1) * sizeof(uint32_t));
  for (int64_t i = J->lo; i < J->hi; ++i) {
    const uint32_t *Li = J->col + J->rp[i];
    int64_t di = (int64_t)(J->rp[i + 1] - J->rp[i]);
    if (J->phase == 0) {
      for (int g = 0; g <= P->W; ++g) {
        uint64_t c = UINT64_MAX;
        if (g == 0) c = row_code(NULL, P, i, Li, di, NULL, 0, 0, scratch);
        else if (g <= i && di > 0 && (J->stride == 0 || (i - g) / J->stride == i / J->stride)) {
          int64_t r = i - g; int64_t dr = (int64_t)(J->rp[r + 1] - J->rp[r]);
          if (dr > 0) c = row_code(NULL, P, i, Li, di, J->col + J->rp[r], dr, g, scratch);
        }
        J->cost[i * (P->W + 1) + g] = c;
      }
    } else {
      int g = J->gsel[i];
      int64_t r = i - g;
      const uint32_t *Lr = g ? J->col + J->rp[r] : NULL;
      int64_t dr = g ? (int64_t)(J->rp[r + 1] - J->rp[r]) : 0;
      row_code(&J->bw, P, i, Li, di, Lr, dr, g, scratch);
    }
  }
  free(scratch);
  return NULL;
}

int bvi_encode(int64_t n, const uint64_t *rowptr, const uint32_t *col, int W, int R, int Lmin, int zk,
               int64_t stride, int nthreads, uint8_t **out, int64_t *nbytes_out, uint8_t *gsel_out) {
  if (n <= 0 || W < 0 || W > 15 || R < 0 || R > 15 || Lmin < 2 || zk < 1 || zk > 8 || nthreads < 1) return -1;
  if (stride < 0 || stride > 0xFFFFFFFFll) return -1;
  for (int64_t i = 0; i < n; ++i) {
    if (rowptr[i + 1] < rowptr[i]) return -1;
    for (uint64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      if ((int64_t)col[k] >= n) return -1;
      if (k > rowptr[i] && col[k] <= col[k - 1]) return -1;
    }
  }
  encp_t P = {W, R, Lmin, zk};
  if (nthreads > 64) nthreads = 64;
  if (n < 4096) nthreads = 1;
  uint64_t *cost = (uint64_t *)malloc((size_t)n * (size_t)(W + 1) * sizeof(uint64_t));
  uint8_t *gsel = (uint8_t *)calloc((size_t)n, 1);
  uint8_t *depth = (uint8_t *)calloc((size_t)n, 1);
  uint64_t *rowbits = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
  enc_job_t jobs[64];
  pthread_t th[64];
  if (!cost || !gsel || !depth || !rowbits) { free(cost); free(gsel); free(depth); free(rowbits); return -2; }
  for (int phase = 0; phase < 2; ++phase) {
    for (int t = 0; t < nthreads; ++t) {
      memset(&jobs[t], 0, sizeof(enc_job_t));
      jobs[t].P = &P; jobs[t].n = n; jobs[t].rp = rowptr; jobs[t].col = col;
      jobs[t].lo = n * t / nthreads; jobs[t].hi = n * (t + 1) / nthreads;
      jobs[t].cost = cost; jobs[t].gsel = gsel; jobs[t].phase = phase; jobs[t].stride = stride;
      pthread_create(&th[t], NULL, enc_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    if (phase == 0) {
      /* sequential choice under the chain-depth bound: fewest bits, ties to
         no reference, then to the nearest reference */
      for (int64_t i = 0; i < n; ++i) {
        int best = 0; uint64_t bc = cost[i * (W + 1)];
        for (int g = 1; g <= W && g <= i; ++g) {
          uint64_t c = cost[i * (W + 1) + g];
          if (c == UINT64_MAX || depth[i - g] >= R) continue;
          if (c < bc) { bc = c; best = g; }
        }
        gsel[i] = (uint8_t)best;
        depth[i] = best ? (uint8_t)(depth[i - best] + 1) : 0;
        rowbits[i] = bc;
      }
    }
  }
  for (int t = 0; t < nthreads; ++t) if (jobs[t].bw.fail) { for (int u = 0; u < nthreads; ++u) free(jobs[u].bw.w); free(cost); free(gsel); free(depth); free(rowbits); return -2; }
  uint64_t body_bits = 0;
  for (int t = 0; t < nthreads; ++t) body_bits += jobs[t].bw.nbits;
  int64_t nseg = stride ? (n + stride - 1) / stride : 0;
  size_t body_words = (size_t)((body_bits + 63) / 64);
  size_t total = 64 + (size_t)nseg * 8 + body_words * 8;
  uint8_t *buf = (uint8_t *)calloc(total, 1);
  if (!buf) { for (int u = 0; u < nthreads; ++u) free(jobs[u].bw.w); free(cost); free(gsel); free(depth); free(rowbits); return -2; }
  uint64_t m = rowptr[n];
  memcpy(buf, "BVMV", 4);
  uint32_t u32;
  u32 = 1; memcpy(buf + 4, &u32, 4);
  memcpy(buf + 8, &n, 8); memcpy(buf + 16, &m, 8);
  u32 = (uint32_t)W; memcpy(buf + 24, &u32, 4);
  u32 = (uint32_t)R; memcpy(buf + 28, &u32, 4);
  u32 = (uint32_t)Lmin; memcpy(buf + 32, &u32, 4);
  u32 = (uint32_t)zk; memcpy(buf + 36, &u32, 4);
  u32 = (uint32_t)stride; memcpy(buf + 40, &u32, 4);
  memcpy(buf + 48, &body_bits, 8);
  memcpy(buf + 56, &nseg, 8);
  /* bit offsets of the segment starts k*S */
  {
    uint64_t off = 0;
    for (int64_t i = 0; i < n; ++i) {
      if (stride && i % stride == 0) memcpy(buf + 64 + 8 * (i / stride), &off, 8);
      off += rowbits[i];
    }
  }
  /* concatenate thread bit buffers (MSB-first words) */
  uint64_t *dst = (uint64_t *)calloc(body_words + 1, sizeof(uint64_t));
  uint64_t pos = 0;
  for (int t = 0; t < nthreads; ++t) {
    bitw_t *b = &jobs[t].bw;
    size_t nw = (size_t)((b->nbits + 63) / 64);
    for (size_t w = 0; w < nw; ++w) {
      uint64_t v = b->w[w];
      int nb = (w + 1 == nw) ? (int)(b->nbits - 64 * w) : 64;
      if (nb < 64) v &= ~((1ull << (64 - nb)) - 1); /* keep top nb bits */
      size_t wi = (size_t)(pos >> 6); int used = (int)(pos & 63);
      dst[wi] |= used ? (v >> used) : v;
      if (used && used + nb > 64) dst[wi + 1] |= v << (64 - used);
      pos += (uint64_t)nb;
    }
    free(b->w);
  }
  /* store words big-endian so the byte stream is MSB-first */
  uint8_t *body = buf + 64 + 8 * nseg;
  for (size_t w = 0; w < body_words; ++w) {
    uint64_t v = dst[w];
    for (int k = 0; k < 8; ++k) body[8 * w + k] = (uint8_t)(v >> (56 - 8 * k));
  }
  free(dst);
  if (gsel_out) memcpy(gsel_out, gsel, (size_t)n);
  free(cost); free(gsel); free(depth); free(rowbits);
  *out = buf; *nbytes_out = (int64_t)total;
  return 0;
}
