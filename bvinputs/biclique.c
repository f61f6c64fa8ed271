/*
 * Biclique decomposition of an adjacency matrix: the input format of the
 * biclique product (Section "Final Remarks" of the paper, after Hernandez and
 * Navarro's biclique extraction).  The edges of G are split into bicliques
 * (S_r, C_r) -- every node of S_r points to every node of C_r -- plus a
 * residual set of edges; a biclique's |S_r| |C_r| edges are stored as the
 * |S_r| + |C_r| ids of its two sets.
 *
 * This file is input production only (like the bitstream encoder in gen.c):
 * it computes no product.  The miner below is this project's own greedy
 * heuristic, not Hernandez and Navarro's clustering algorithm; any edge
 * partition is a valid input, and the miner only has to produce one that
 * saves words on graphs with the copy structure of the web-like generator.
 *
 * Miner.  Rows are taken in order.  Row i, with its edges not yet assigned
 * (list R_i), seeds S = {i}, C = R_i, and grows S greedily from the rows
 * i+1 .. i+window: the candidate j whose remaining list shares the most ids
 * with C (ties: smallest j) joins while the saving
 *     gain(S, C) = |S| |C| - |S| - |C|
 * grows (C shrinks to C & R_j).  A biclique with |S| >= 2, |C| >= cmin and
 * gain > 0 is emitted and its edges are removed from the lists of S's rows;
 * row i then seeds again until no biclique is found.  Whatever remains is
 * the residual.  Rows are mined in independent blocks of `block` rows
 * (candidates stay inside the block), one block per worker thread at a time,
 * and the blocks' outputs are concatenated in row order, so the result does
 * not depend on the thread count.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  uint32_t *a;
  size_t n, cap;
} vec32;

static int v_push(vec32 *v, uint32_t x) {
  if (v->n == v->cap) {
    size_t nc = v->cap ? 2 * v->cap : 64;
    uint32_t *p = (uint32_t *)realloc(v->a, nc * sizeof(uint32_t));
    if (!p) return -1;
    v->a = p;
    v->cap = nc;
  }
  v->a[v->n++] = x;
  return 0;
}

typedef struct {
  vec32 s, c, s_len, c_len;  /* bicliques: ids of S and C, and the set sizes */
  vec32 res_col, res_len;    /* residual edges of each row of the block */
  int err;
} mine_out;

typedef struct {
  const uint64_t *rowptr;
  const uint32_t *col;
  int64_t n, block;
  int window, cmin;
  mine_out *outs;
  int64_t nblocks;
  int64_t next;
  pthread_mutex_t mu;
} mine_ctx;

/* |a & b| of two sorted lists */
static size_t inter_count(const uint32_t *a, size_t na, const uint32_t *b, size_t nb) {
  size_t i = 0, j = 0, k = 0;
  while (i < na && j < nb) {
    if (a[i] < b[j]) ++i;
    else if (a[i] > b[j]) ++j;
    else { ++k; ++i; ++j; }
  }
  return k;
}
/* a <- a & b, returns the new length */
static size_t inter_into(uint32_t *a, size_t na, const uint32_t *b, size_t nb) {
  size_t i = 0, j = 0, k = 0;
  while (i < na && j < nb) {
    if (a[i] < b[j]) ++i;
    else if (a[i] > b[j]) ++j;
    else { a[k++] = a[i]; ++i; ++j; }
  }
  return k;
}
/* a <- a \ b, returns the new length */
static size_t minus_into(uint32_t *a, size_t na, const uint32_t *b, size_t nb) {
  size_t i = 0, j = 0, k = 0;
  while (i < na) {
    while (j < nb && b[j] < a[i]) ++j;
    if (j < nb && b[j] == a[i]) { ++i; ++j; continue; }
    a[k++] = a[i++];
  }
  return k;
}

static int64_t gain(int64_t s, int64_t c) { return s * c - s - c; }

static void mine_block(const mine_ctx *ctx, int64_t b, mine_out *o) {
  const int64_t r0 = b * ctx->block;
  const int64_t r1 = r0 + ctx->block < ctx->n ? r0 + ctx->block : ctx->n;
  const int64_t nr = r1 - r0;
  /* remaining lists of the block's rows: copies, shrunk in place */
  const uint64_t base = ctx->rowptr[r0];
  const size_t tot = (size_t)(ctx->rowptr[r1] - base);
  uint32_t *buf = (uint32_t *)malloc((tot ? tot : 1) * sizeof(uint32_t));
  size_t *len = (size_t *)malloc((size_t)(nr ? nr : 1) * sizeof(size_t));
  uint32_t *C = (uint32_t *)malloc((tot ? tot : 1) * sizeof(uint32_t));
  int64_t *S = (int64_t *)malloc((size_t)(ctx->window + 1) * sizeof(int64_t));
  char *inS = (char *)calloc((size_t)(ctx->window + 1), 1);
  if (!buf || !len || !C || !S || !inS) { o->err = 1; goto done; }
  if (tot) memcpy(buf, ctx->col + base, tot * sizeof(uint32_t));
  for (int64_t r = 0; r < nr; ++r) len[r] = (size_t)(ctx->rowptr[r0 + r + 1] - ctx->rowptr[r0 + r]);
#define ROW(r) (buf + (ctx->rowptr[r0 + (r)] - base))
  for (int64_t i = 0; i < nr; ++i) {
    for (;;) {
      if (len[i] < (size_t)ctx->cmin) break;
      size_t nc = len[i];
      memcpy(C, ROW(i), nc * sizeof(uint32_t));
      int ns = 1;
      S[0] = i;
      const int64_t jmax = i + ctx->window < nr - 1 ? i + ctx->window : nr - 1;
      memset(inS, 0, (size_t)(ctx->window + 1));
      for (;;) {
        int64_t best = -1;
        size_t bestc = 0;
        for (int64_t j = i + 1; j <= jmax; ++j) {
          if (inS[j - i] || len[j] == 0) continue;
          const size_t k = inter_count(C, nc, ROW(j), len[j]);
          if (k > bestc) { bestc = k; best = j; }
        }
        if (best < 0 || gain(ns + 1, (int64_t)bestc) <= gain(ns, (int64_t)nc)) break;
        nc = inter_into(C, nc, ROW(best), len[best]);
        S[ns++] = best;
        inS[best - i] = 1;
      }
      if (ns < 2 || nc < (size_t)ctx->cmin || gain(ns, (int64_t)nc) <= 0) break;
      /* emit; S in ascending row order */
      for (int a = 1; a < ns; ++a)
        for (int q = a; q > 0 && S[q - 1] > S[q]; --q) { int64_t t = S[q]; S[q] = S[q - 1]; S[q - 1] = t; }
      for (int a = 0; a < ns; ++a) {
        if (v_push(&o->s, (uint32_t)(r0 + S[a]))) { o->err = 1; goto done; }
        len[S[a]] = minus_into(ROW(S[a]), len[S[a]], C, nc);
      }
      for (size_t a = 0; a < nc; ++a)
        if (v_push(&o->c, C[a])) { o->err = 1; goto done; }
      if (v_push(&o->s_len, (uint32_t)ns) || v_push(&o->c_len, (uint32_t)nc)) { o->err = 1; goto done; }
    }
  }
  for (int64_t r = 0; r < nr; ++r) {
    for (size_t a = 0; a < len[r]; ++a)
      if (v_push(&o->res_col, ROW(r)[a])) { o->err = 1; goto done; }
    if (v_push(&o->res_len, (uint32_t)len[r])) { o->err = 1; goto done; }
  }
#undef ROW
done:
  free(buf);
  free(len);
  free(C);
  free(S);
  free(inS);
}

static void *mine_worker(void *arg) {
  mine_ctx *ctx = (mine_ctx *)arg;
  for (;;) {
    pthread_mutex_lock(&ctx->mu);
    const int64_t b = ctx->next++;
    pthread_mutex_unlock(&ctx->mu);
    if (b >= ctx->nblocks) break;
    mine_block(ctx, b, &ctx->outs[b]);
  }
  return NULL;
}

/* Mine a biclique decomposition of the CSR graph (rows strictly increasing).
 * Outputs (malloc'ed, freed with bvi_free): nbic bicliques, S of biclique r =
 * sidx[sptr[r] .. sptr[r+1]), C of biclique r = cidx[cptr[r] .. cptr[r+1]),
 * both ascending; the residual as CSR rptr (n+1), rcol (ascending per row).
 * Returns 0, or -1 on bad arguments / allocation failure. */
int bvi_biclique_mine(int64_t n, const uint64_t *rowptr, const uint32_t *col, int window, int cmin, int64_t block,
                      int nthreads, int64_t *nbic, uint64_t **sptr, uint32_t **sidx, uint64_t **cptr,
                      uint32_t **cidx, uint64_t **rptr, uint32_t **rcol) {
  if (n < 1 || !rowptr || window < 1 || window > 1024 || cmin < 1 || block < 1 || !nbic || !sptr || !sidx ||
      !cptr || !cidx || !rptr || !rcol)
    return -1;
  mine_ctx ctx;
  ctx.rowptr = rowptr;
  ctx.col = col;
  ctx.n = n;
  ctx.block = block;
  ctx.window = window;
  ctx.cmin = cmin;
  ctx.nblocks = (n + block - 1) / block;
  ctx.next = 0;
  ctx.outs = (mine_out *)calloc((size_t)ctx.nblocks, sizeof(mine_out));
  if (!ctx.outs) return -1;
  pthread_mutex_init(&ctx.mu, NULL);
  int nt = nthreads < 1 ? 1 : (nthreads > 64 ? 64 : nthreads);
  if (nt > ctx.nblocks) nt = (int)ctx.nblocks;
  pthread_t th[64];
  int started = 0;
  for (int t = 1; t < nt; ++t)
    if (pthread_create(&th[started], NULL, mine_worker, &ctx) == 0) ++started;
  mine_worker(&ctx);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  pthread_mutex_destroy(&ctx.mu);
  int rc = 0;
  size_t nb = 0, ns = 0, nc = 0, nres = 0;
  for (int64_t b = 0; b < ctx.nblocks; ++b) {
    if (ctx.outs[b].err) rc = -1;
    nb += ctx.outs[b].s_len.n;
    ns += ctx.outs[b].s.n;
    nc += ctx.outs[b].c.n;
    nres += ctx.outs[b].res_col.n;
  }
  uint64_t *sp = NULL, *cp = NULL, *rp = NULL;
  uint32_t *si = NULL, *ci = NULL, *rc_ = NULL;
  if (rc == 0) {
    sp = (uint64_t *)malloc((nb + 1) * sizeof(uint64_t));
    cp = (uint64_t *)malloc((nb + 1) * sizeof(uint64_t));
    rp = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
    si = (uint32_t *)malloc((ns ? ns : 1) * sizeof(uint32_t));
    ci = (uint32_t *)malloc((nc ? nc : 1) * sizeof(uint32_t));
    rc_ = (uint32_t *)malloc((nres ? nres : 1) * sizeof(uint32_t));
    if (!sp || !cp || !rp || !si || !ci || !rc_) rc = -1;
  }
  if (rc == 0) {
    size_t kb = 0, ks = 0, kc = 0, kr = 0;
    int64_t row = 0;
    sp[0] = cp[0] = rp[0] = 0;
    for (int64_t b = 0; b < ctx.nblocks; ++b) {
      const mine_out *o = &ctx.outs[b];
      memcpy(si + ks, o->s.a, o->s.n * sizeof(uint32_t));
      memcpy(ci + kc, o->c.a, o->c.n * sizeof(uint32_t));
      memcpy(rc_ + kr, o->res_col.a, o->res_col.n * sizeof(uint32_t));
      for (size_t q = 0; q < o->s_len.n; ++q) {
        sp[kb + 1] = sp[kb] + o->s_len.a[q];
        cp[kb + 1] = cp[kb] + o->c_len.a[q];
        ++kb;
      }
      for (size_t q = 0; q < o->res_len.n; ++q, ++row) rp[row + 1] = rp[row] + o->res_len.a[q];
      ks += o->s.n;
      kc += o->c.n;
      kr += o->res_col.n;
    }
    *nbic = (int64_t)nb;
    *sptr = sp;
    *cptr = cp;
    *sidx = si;
    *cidx = ci;
    *rptr = rp;
    *rcol = rc_;
  } else {
    free(sp); free(cp); free(rp); free(si); free(ci); free(rc_);
  }
  for (int64_t b = 0; b < ctx.nblocks; ++b) {
    free(ctx.outs[b].s.a); free(ctx.outs[b].c.a); free(ctx.outs[b].s_len.a);
    free(ctx.outs[b].c_len.a); free(ctx.outs[b].res_col.a); free(ctx.outs[b].res_len.a);
  }
  free(ctx.outs);
  return rc;
}
