/*
 * kp_oracle.c -- plain, slow, obviously-correct CPU oracle for the per-user
 * subproblem sweep of the Lagrangian-dual knapsack solver
 * (Zhang, Qi, Hua, Yang: "Solving Billion-Scale Knapsack Problems", WWW'20).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The GPU product path
 * never calls it and shares no code with it.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * (no FMA contraction: every a - b*c below is two separately rounded operations).
 *
 * Every function follows one passage of the paper, cited in its comment.
 * Readings of points the paper leaves open are marked "Reading:".
 * OpenMP is used across users only; every per-user computation is sequential
 * and in a fixed order, and sums across users are combined in fixed chunks, so
 * results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int64_t N;
  int32_t M, K;
  const float *p;               /* [N*M] */
  int32_t b_format;             /* 0 = dense, 1 = per-item CSR */
  const float *b;               /* dense [N*M*K], k fastest */
  const int64_t *rowptr;        /* CSR [N*M+1] */
  const int32_t *col;           /* CSR columns, ascending per item */
  const float *val;             /* CSR values */
  const double *B;              /* [K] budgets */
  int32_t L;                    /* local-constraint forest */
  const int32_t *parent;        /* [L], -1 = root */
  const int32_t *cap;           /* [L] */
  const int32_t *leaf_of_item;  /* [M], innermost node holding j, or -1 */
} orc_problem;

#define MAXM 64
#define CHUNK 4096

/* ------------------------------------------------------------------------ */
/* Local constraints as explicit sets S_l with caps C_l (Eq.3), visited in a  */
/* topological order of the containment DAG (Sec. 2.1): subsets before       */
/* supersets.  Reading: |S_l| ascending, then node id.                       */
/* ------------------------------------------------------------------------ */
typedef struct {
  int L, M;
  unsigned char *in;   /* [L*M] membership */
  int *size;           /* [L] */
  int *topo;           /* [L] node ids in topological order */
  const int32_t *cap;
} orc_sets;

static void sets_build(const orc_problem *pr, orc_sets *s) {
  int L = pr->L, M = pr->M;
  s->L = L; s->M = M; s->cap = pr->cap;
  s->in = (unsigned char *)calloc((size_t)(L > 0 ? L : 1) * M, 1);
  s->size = (int *)calloc(L > 0 ? L : 1, sizeof(int));
  s->topo = (int *)calloc(L > 0 ? L : 1, sizeof(int));
  for (int j = 0; j < M; ++j) {
    for (int l = pr->leaf_of_item[j]; l >= 0; l = pr->parent[l]) {
      s->in[(size_t)l * M + j] = 1;
    }
  }
  for (int l = 0; l < L; ++l) {
    int c = 0;
    for (int j = 0; j < M; ++j) c += s->in[(size_t)l * M + j];
    s->size[l] = c;
    s->topo[l] = l;
  }
  /* insertion sort of node ids by (size asc, id asc) */
  for (int a = 1; a < L; ++a) {
    int v = s->topo[a], b = a - 1;
    while (b >= 0 && (s->size[s->topo[b]] > s->size[v])) { s->topo[b + 1] = s->topo[b]; --b; }
    s->topo[b + 1] = v;
  }
}

static void sets_free(orc_sets *s) { free(s->in); free(s->size); free(s->topo); }

/* ------------------------------------------------------------------------ */
/* Cost-adjusted profit (Sec. 4.2):  p~_ij = p_ij - sum_k lambda_k b_ijk.    */
/* FP64, k ascending, one rounding for the product and one for the          */
/* subtraction.  CSR visits its stored columns in ascending order.           */
/* ------------------------------------------------------------------------ */
static void score_user(const orc_problem *pr, const double *lam, int64_t i, double *pt) {
  int M = pr->M, K = pr->K;
  for (int j = 0; j < M; ++j) {
    int64_t r = i * M + j;
    double acc = (double)pr->p[r];
    if (pr->b_format == 0) {
      const float *bb = pr->b + r * K;
      for (int k = 0; k < K; ++k) {
        double prod = lam[k] * (double)bb[k];
        acc = acc - prod;
      }
    } else {
      for (int64_t e = pr->rowptr[r]; e < pr->rowptr[r + 1]; ++e) {
        double prod = lam[pr->col[e]] * (double)pr->val[e];
        acc = acc - prod;
      }
    }
    pt[j] = acc;
  }
}

/* b_ijk for one item row (dense or CSR) */
static double b_at(const orc_problem *pr, int64_t r, int k) {
  if (pr->b_format == 0) return (double)pr->b[r * pr->K + k];
  for (int64_t e = pr->rowptr[r]; e < pr->rowptr[r + 1]; ++e)
    if (pr->col[e] == k) return (double)pr->val[e];
  return 0.0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 (Sec. 4.2): greedy for hierarchical local constraints.        */
/*  1. x_j = 1 iff the adjusted profit is strictly positive;                 */
/*  2. order the items by adjusted profit, non-increasing                    */
/*     (Reading: ties go to the lower item index -- a stable sort);          */
/*  3. for every set S_l in topological order, among its still-selected      */
/*     members keep the first C_l in that order and deselect the rest.       */
/* ------------------------------------------------------------------------ */
static void alg1(const orc_sets *s, const double *z, unsigned char *x) {
  int M = s->M;
  int order[MAXM];
  for (int j = 0; j < M; ++j) { x[j] = z[j] > 0.0; order[j] = j; }
  for (int a = 1; a < M; ++a) {       /* stable insertion sort, z descending */
    int v = order[a], b = a - 1;
    while (b >= 0 && z[order[b]] < z[v]) { order[b + 1] = order[b]; --b; }
    order[b + 1] = v;
  }
  for (int t = 0; t < s->L; ++t) {
    int l = s->topo[t], kept = 0;
    const unsigned char *in = s->in + (size_t)l * M;
    for (int a = 0; a < M; ++a) {
      int j = order[a];
      if (!in[j] || !x[j]) continue;
      if (kept < s->cap[l]) ++kept; else x[j] = 0;
    }
  }
}

/* Neumaier-compensated running sum */
typedef struct { double s, c; } nsum;
static inline void nadd(nsum *a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v; else a->c += (v - t) + a->s;
  a->s = t;
}
static inline double nval(const nsum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* Exact sums of doubles.  Reading: the reduce of Alg.4 compares the total   */
/* resource a threshold lets through with B_k -- a sum of real numbers -- so */
/* the oracle forms it exactly: a two's-complement fixed-point integer whose */
/* lowest bit is 2^-1088 (below every double, subnormals included) and whose */
/* 34 limbs of 64 bits reach 2^1087 (every double, with room for the sum of  */
/* up to 2^63 of them).  Adding a double places its 53-bit significand at    */
/* its binary position and propagates the carry (or the borrow).             */
/* ------------------------------------------------------------------------ */
#define XLIMBS 34
#define XLSB 1088
typedef struct { uint64_t w[XLIMBS]; } xsum;

static void xsum_zero(xsum *a) { memset(a->w, 0, sizeof a->w); }

static void xsum_add(xsum *a, double v) {
  if (v == 0.0) return;
  int e;
  double fr = frexp(fabs(v), &e);                    /* |v| = fr * 2^e, fr in [0.5, 1) */
  uint64_t m = (uint64_t)ldexp(fr, 53);              /* |v| = m * 2^(e - 53), exact */
  int pos = e - 53 + XLSB;                           /* bit position of m's lowest bit */
  if (pos < 0) { m >>= -pos; pos = 0; }              /* subnormals: the dropped bits are zero */
  int limb = pos / 64, sh = pos % 64;
  uint64_t lo = m << sh, hi = sh ? m >> (64 - sh) : 0;
  if (v > 0.0) {
    uint64_t c;
    uint64_t t = a->w[limb] + lo;
    c = t < lo;
    a->w[limb] = t;
    for (int i = limb + 1; i < XLIMBS && (c || (i == limb + 1 && hi)); ++i) {
      uint64_t add = (i == limb + 1) ? hi : 0;
      uint64_t u = a->w[i] + add;
      uint64_t c1 = u < add;
      uint64_t u2 = u + c;
      uint64_t c2 = u2 < c;
      a->w[i] = u2;
      c = c1 | c2;
    }
  } else {
    uint64_t b;
    uint64_t t = a->w[limb] - lo;
    b = a->w[limb] < lo;
    a->w[limb] = t;
    for (int i = limb + 1; i < XLIMBS && (b || (i == limb + 1 && hi)); ++i) {
      uint64_t sub = (i == limb + 1) ? hi : 0;
      uint64_t u = a->w[i] - sub;
      uint64_t b1 = a->w[i] < sub;
      uint64_t u2 = u - b;
      uint64_t b2 = u < b;
      a->w[i] = u2;
      b = b1 | b2;
    }
  }
}

/* sign of (a - v): -1, 0 or 1 */
static int xsum_cmp(const xsum *a, double v) {
  xsum d = *a;
  xsum_add(&d, -v);
  if (d.w[XLIMBS - 1] >> 63) return -1;
  for (int i = 0; i < XLIMBS; ++i)
    if (d.w[i]) return 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Dual evaluation at lambda (Eq.5 and Alg.2 Map/Reduce):                     */
/*  x_i = Alg1(p~_i); v_ik = sum_j b_ijk x_ij (j ascending);                  */
/*  R_k = sum_i v_ik; P = sum p x; G_i = sum_j p~_ij x_ij;                    */
/*  g(lambda) = sum_i G_i + sum_k lambda_k B_k.                               */
/* Outputs: x [N*M] (uint8, optional), R [K], g, P, G [N] (optional).         */
/* Returns 0, or -1 when M exceeds the oracle's limit.                        */
/* ------------------------------------------------------------------------ */
int orc_eval(const orc_problem *pr, const double *lam, unsigned char *x_out, double *R_out,
             double *g_out, double *P_out, double *G_out) {
  if (pr->M > MAXM) return -1;
  int M = pr->M, K = pr->K;
  int64_t N = pr->N, nchunk = (N + CHUNK - 1) / CHUNK;
  orc_sets s; sets_build(pr, &s);
  nsum *part = (nsum *)calloc((size_t)(nchunk > 0 ? nchunk : 1) * (K + 2), sizeof(nsum));
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t ch = 0; ch < nchunk; ++ch) {
    nsum *ps = part + ch * (K + 2);
    double pt[MAXM]; unsigned char x[MAXM];
    double *v = (double *)malloc(sizeof(double) * (size_t)K);
    for (int64_t i = ch * CHUNK; i < N && i < (ch + 1) * CHUNK; ++i) {
      score_user(pr, lam, i, pt);
      alg1(&s, pt, x);
      for (int k = 0; k < K; ++k) v[k] = 0.0;
      double Pi = 0.0, Gi = 0.0;
      for (int j = 0; j < M; ++j) {
        int64_t r = i * M + j;
        if (x_out) x_out[r] = x[j];
        if (!x[j]) continue;
        Pi = Pi + (double)pr->p[r];
        Gi = Gi + pt[j];
        if (pr->b_format == 0) {
          for (int k = 0; k < K; ++k) v[k] = v[k] + (double)pr->b[r * K + k];
        } else {
          for (int64_t e = pr->rowptr[r]; e < pr->rowptr[r + 1]; ++e)
            v[pr->col[e]] = v[pr->col[e]] + (double)pr->val[e];
        }
      }
      if (G_out) G_out[i] = Gi;
      for (int k = 0; k < K; ++k) nadd(&ps[k], v[k]);
      nadd(&ps[K], Gi);
      nadd(&ps[K + 1], Pi);
    }
    free(v);
  }
  nsum tot[2] = {{0, 0}, {0, 0}};
  for (int k = 0; k < K; ++k) {
    nsum a = {0, 0};
    for (int64_t ch = 0; ch < nchunk; ++ch) nadd(&a, nval(&part[ch * (K + 2) + k]));
    R_out[k] = nval(&a);
  }
  for (int64_t ch = 0; ch < nchunk; ++ch) {
    nadd(&tot[0], nval(&part[ch * (K + 2) + K]));
    nadd(&tot[1], nval(&part[ch * (K + 2) + K + 1]));
  }
  for (int k = 0; k < K; ++k) nadd(&tot[0], lam[k] * pr->B[k]);
  *g_out = nval(&tot[0]);
  *P_out = nval(&tot[1]);
  free(part);
  sets_free(&s);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Dual descent step, Eq.(14):  lambda_k <- max(lambda_k + alpha (R_k - B_k), 0). */
/* ------------------------------------------------------------------------ */
void orc_dd_update(int K, double alpha, const double *R, const double *B, double *lam) {
  for (int k = 0; k < K; ++k) {
    double d = R[k] - B[k];
    double st = alpha * d;
    double nl = lam[k] + st;
    lam[k] = nl > 0.0 ? nl : 0.0;
  }
}

/* ------------------------------------------------------------------------ */
/* SCD Map for one user and one coordinate k (Alg.3 + Alg.4 Map).             */
/* Lines z_j(lam_k) = c_j - lam_k b_jk.  Reading: c_j = p~_j + lam_k^t b_jk    */
/* (adding back the k-th term of the score, one FP64 product and one add).   */
/* Alg.3 candidates: lam with z_j = 0 (b_jk > 0), and lam with z_j = z_j'    */
/* (b_jk != b_j'k), computed as c_j/b_j and (c_j - c_j')/(b_j - b_j');        */
/* only finite values > 0 are kept (lambda >= 0, Eq.10), duplicates removed. */
/* Alg.4 Map: walk the candidates in decreasing order; Reading: the          */
/* consumption attributed to candidate u_r is evaluated strictly below it,   */
/* at the midpoint (u_r + u_{r+1})/2 (u_m/2 for the last one), so that the   */
/* greedy never sees the tie that sits exactly at u_r.  Emit                 */
/* (v1 = u_r, v2 = current - previous) when consumption rises; previous is   */
/* updated inside the If, as printed.                                        */
/* Writes up to cap pairs; returns the number of pairs (may exceed cap).     */
/* ------------------------------------------------------------------------ */
static int cmp_desc(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x < y) - (x > y);
}

static int scd_map_user_k(const orc_problem *pr, const orc_sets *s, const double *lam, int64_t i,
                          int k, const double *pt, double *v1, double *v2, int cap_out,
                          double *cand /* scratch [M + M(M-1)/2] */) {
  int M = pr->M;
  double c[MAXM], bk[MAXM], z[MAXM];
  unsigned char x[MAXM];
  for (int j = 0; j < M; ++j) {
    bk[j] = b_at(pr, i * M + j, k);
    double add = lam[k] * bk[j];
    c[j] = pt[j] + add;
  }
  int m = 0;
  for (int j = 0; j < M; ++j) {
    if (bk[j] > 0.0) {
      double u = c[j] / bk[j];
      if (isfinite(u) && u > 0.0) cand[m++] = u;
    }
    for (int jj = j + 1; jj < M; ++jj) {
      if (bk[j] != bk[jj]) {
        double num = c[j] - c[jj];
        double den = bk[j] - bk[jj];
        double u = num / den;
        if (isfinite(u) && u > 0.0) cand[m++] = u;
      }
    }
  }
  qsort(cand, (size_t)m, sizeof(double), cmp_desc);
  int mu = 0;
  for (int a = 0; a < m; ++a)
    if (mu == 0 || cand[a] != cand[mu - 1]) cand[mu++] = cand[a];
  double prev = 0.0;
  int ne = 0;
  for (int r = 0; r < mu; ++r) {
    double t = (r + 1 < mu) ? (cand[r] + cand[r + 1]) * 0.5 : cand[r] * 0.5;
    for (int j = 0; j < M; ++j) {
      double prod = t * bk[j];
      z[j] = c[j] - prod;
    }
    alg1(s, z, x);
    double cur = 0.0;
    for (int j = 0; j < M; ++j)
      if (x[j]) cur = cur + bk[j];
    if (cur > prev) {
      if (ne < cap_out) { v1[ne] = cand[r]; v2[ne] = cur - prev; }
      ++ne;
      prev = cur;
    }
  }
  return ne;
}

/* Emitted pairs of users [u0,u1) for every k: pairs are written in the order   */
/* (user ascending, k ascending, emission order).  kk/uu record k and user.    */
/* Returns the number of pairs (writes at most cap).                           */
int64_t orc_scd_map(const orc_problem *pr, const double *lam, int64_t u0, int64_t u1,
                    int32_t *kk, int64_t *uu, double *v1, double *v2, int64_t cap) {
  if (pr->M > MAXM) return -1;
  int M = pr->M, K = pr->K;
  orc_sets s; sets_build(pr, &s);
  int maxc = M + M * (M - 1) / 2 + 1;
  double *cand = (double *)malloc(sizeof(double) * maxc);
  double *a = (double *)malloc(sizeof(double) * maxc), *b = (double *)malloc(sizeof(double) * maxc);
  double pt[MAXM];
  int64_t n = 0;
  for (int64_t i = u0; i < u1; ++i) {
    score_user(pr, lam, i, pt);
    for (int k = 0; k < K; ++k) {
      int ne = scd_map_user_k(pr, &s, lam, i, k, pt, a, b, maxc, cand);
      for (int e = 0; e < ne; ++e, ++n) {
        if (n < cap) { kk[n] = k; uu[n] = i; v1[n] = a[e]; v2[n] = b[e]; }
      }
    }
  }
  free(cand); free(a); free(b);
  sets_free(&s);
  return n;
}

/* ------------------------------------------------------------------------ */
/* SCD Reduce for one k (Alg.4 Reduce).  Return 0 when the total increment   */
/* sum v2 fits in B_k.  Otherwise, Reading: walk the distinct v1 values in   */
/* decreasing order with the running sum of v2 (including the value itself) */
/* and return the first v1 at which that sum exceeds B_k -- the smallest    */
/* lambda_k at which consumption just above it still fits the budget.  The  */
/* sums are exact (xsum), so the threshold does not depend on their order.   */
/* The pairs are sorted in place (v1 descending).                            */
/* ------------------------------------------------------------------------ */
typedef struct { double v1, v2; } pair_t;
static int cmp_pair_desc(const void *a, const void *b) {
  double x = ((const pair_t *)a)->v1, y = ((const pair_t *)b)->v1;
  return (x < y) - (x > y);
}

double orc_scd_reduce(int64_t n, double *v1, double *v2, double Bk) {
  xsum total;
  xsum_zero(&total);
  for (int64_t e = 0; e < n; ++e) xsum_add(&total, v2[e]);
  if (xsum_cmp(&total, Bk) <= 0) return 0.0;
  pair_t *pp = (pair_t *)malloc(sizeof(pair_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t e = 0; e < n; ++e) { pp[e].v1 = v1[e]; pp[e].v2 = v2[e]; }
  qsort(pp, (size_t)n, sizeof(pair_t), cmp_pair_desc);
  xsum cum;
  xsum_zero(&cum);
  double ans = pp[n - 1].v1;
  int64_t e = 0;
  while (e < n) {
    double v = pp[e].v1;
    while (e < n && pp[e].v1 == v) { xsum_add(&cum, pp[e].v2); ++e; }
    if (xsum_cmp(&cum, Bk) > 0) { ans = v; break; }
  }
  for (int64_t q = 0; q < n; ++q) { v1[q] = pp[q].v1; v2[q] = pp[q].v2; }
  free(pp);
  return ans;
}

/* One full SCD iteration (Alg.4): Map over all users, Reduce per k,          */
/* synchronous update of every coordinate from the same lambda^t.            */
/* Returns 0, -1 on M overflow, -2 on allocation failure.                    */
int orc_scd_sweep_mask(const orc_problem *pr, const double *lam_in, double *lam_out,
                       const unsigned char *kmask);
int orc_scd_sweep(const orc_problem *pr, const double *lam_in, double *lam_out) {
  return orc_scd_sweep_mask(pr, lam_in, lam_out, NULL);
}

/* Same, restricted to the coordinates with kmask[k] != 0 (cyclic and block
   CD, Sec. 4.3.2); the other coordinates are copied from lam_in. */
int orc_scd_sweep_mask(const orc_problem *pr, const double *lam_in, double *lam_out,
                       const unsigned char *kmask) {
  if (pr->M > MAXM) return -1;
  int M = pr->M, K = pr->K;
  int64_t N = pr->N;
  int64_t nchunk = (N + CHUNK - 1) / CHUNK;
  int maxc = M + M * (M - 1) / 2 + 1;
  /* per-chunk pair lists, gathered in chunk order */
  int64_t *cnt = (int64_t *)calloc((size_t)(nchunk > 0 ? nchunk : 1), sizeof(int64_t));
  int32_t **ck = (int32_t **)calloc((size_t)(nchunk > 0 ? nchunk : 1), sizeof(void *));
  double **c1 = (double **)calloc((size_t)(nchunk > 0 ? nchunk : 1), sizeof(void *));
  double **c2 = (double **)calloc((size_t)(nchunk > 0 ? nchunk : 1), sizeof(void *));
  int fail = 0;
  orc_sets s; sets_build(pr, &s);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t ch = 0; ch < nchunk; ++ch) {
    int64_t cap = 1024, n = 0;
    int32_t *kk = (int32_t *)malloc(sizeof(int32_t) * cap);
    double *a1 = (double *)malloc(sizeof(double) * cap), *a2 = (double *)malloc(sizeof(double) * cap);
    double *cand = (double *)malloc(sizeof(double) * maxc);
    double *t1 = (double *)malloc(sizeof(double) * maxc), *t2 = (double *)malloc(sizeof(double) * maxc);
    double pt[MAXM];
    for (int64_t i = ch * CHUNK; i < N && i < (ch + 1) * CHUNK; ++i) {
      score_user(pr, lam_in, i, pt);
      for (int k = 0; k < K; ++k) {
        if (kmask && !kmask[k]) continue;
        int ne = scd_map_user_k(pr, &s, lam_in, i, k, pt, t1, t2, maxc, cand);
        if (n + ne > cap) {
          while (n + ne > cap) cap *= 2;
          kk = (int32_t *)realloc(kk, sizeof(int32_t) * cap);
          a1 = (double *)realloc(a1, sizeof(double) * cap);
          a2 = (double *)realloc(a2, sizeof(double) * cap);
          if (!kk || !a1 || !a2) { fail = 1; break; }
        }
        for (int e = 0; e < ne; ++e, ++n) { kk[n] = k; a1[n] = t1[e]; a2[n] = t2[e]; }
      }
    }
    cnt[ch] = n; ck[ch] = kk; c1[ch] = a1; c2[ch] = a2;
    free(cand); free(t1); free(t2);
  }
  if (!fail) {
    int64_t *per = (int64_t *)calloc((size_t)K, sizeof(int64_t));
    for (int64_t ch = 0; ch < nchunk; ++ch)
      for (int64_t e = 0; e < cnt[ch]; ++e) per[ck[ch][e]]++;
    for (int k = 0; k < K; ++k) {
      if (kmask && !kmask[k]) { lam_out[k] = lam_in[k]; continue; }
      double *v1 = (double *)malloc(sizeof(double) * (size_t)(per[k] + 1));
      double *v2 = (double *)malloc(sizeof(double) * (size_t)(per[k] + 1));
      int64_t n = 0;
      for (int64_t ch = 0; ch < nchunk; ++ch)
        for (int64_t e = 0; e < cnt[ch]; ++e)
          if (ck[ch][e] == k) { v1[n] = c1[ch][e]; v2[n] = c2[ch][e]; ++n; }
      lam_out[k] = orc_scd_reduce(n, v1, v2, pr->B[k]);
      free(v1); free(v2);
    }
    free(per);
  }
  for (int64_t ch = 0; ch < nchunk; ++ch) { free(ck[ch]); free(c1[ch]); free(c2[ch]); }
  free(cnt); free(ck); free(c1); free(c2);
  sets_free(&s);
  return fail ? -2 : 0;
}

/* ------------------------------------------------------------------------ */
/* Consumption of knapsack k over users [u0,u1) when only lambda_k is moved   */
/* to `value' (the aggregate step function the SCD Reduce thresholds), using */
/* the same lines c_j - value*b_jk as the Map.  Used to check coordinate      */
/* optimality of a threshold at any instance size.                            */
/* ------------------------------------------------------------------------ */
double orc_consumption_at(const orc_problem *pr, const double *lam, int k, double value,
                          int64_t u0, int64_t u1) {
  if (pr->M > MAXM) return -1.0;
  int M = pr->M;
  int64_t nchunk = (u1 - u0 + CHUNK - 1) / CHUNK;
  orc_sets s; sets_build(pr, &s);
  double *part = (double *)calloc((size_t)(nchunk > 0 ? nchunk : 1), sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t ch = 0; ch < nchunk; ++ch) {
    double pt[MAXM], z[MAXM], bk[MAXM];
    unsigned char x[MAXM];
    double acc = 0.0;
    for (int64_t i = u0 + ch * CHUNK; i < u1 && i < u0 + (ch + 1) * CHUNK; ++i) {
      score_user(pr, lam, i, pt);
      for (int j = 0; j < M; ++j) {
        bk[j] = b_at(pr, i * M + j, k);
        double add = lam[k] * bk[j];
        double c = pt[j] + add;
        double prod = value * bk[j];
        z[j] = c - prod;
      }
      alg1(&s, z, x);
      for (int j = 0; j < M; ++j)
        if (x[j]) acc = acc + bk[j];
    }
    part[ch] = acc;
  }
  double tot = 0.0;
  for (int64_t ch = 0; ch < nchunk; ++ch) tot = tot + part[ch];
  free(part);
  sets_free(&s);
  return tot;
}

/* ------------------------------------------------------------------------ */
/* Post-processing for feasibility (Sec. 5.4).                                */
/* Group dual value p~_i = sum_j p_ij x_ij - sum_k lambda_k sum_j b_ijk x_ij  */
/* (= G_i).  Users are ordered by (p~_i ascending, i ascending) and reset to  */
/* x_i = 0 one by one until every R_k <= B_k.                                 */
/* mode 0 (Reading adopted): only users that consume at least one knapsack   */
/*   violated at the start are walked; the shortest prefix of that ordered   */
/*   list that brings every violated k within budget is reset.               */
/* mode 1 (literal): every user is walked in that order.                     */
/* A violated knapsack counts as covered once its total consumption minus    */
/* the reset users' consumption, both exact sums (xsum), is at most B_k: the  */
/* consumption a reset leaves is a real number (reading A24 applied to Sec.  */
/* 5.4), so the reset set does not depend on a summation order.              */
/* Outputs: x [N*M] after reset (optional), P, R [K], the reset count, and   */
/* the reset users in reset order (optional, up to cap).                     */
/* ------------------------------------------------------------------------ */
typedef struct { double key; int64_t i; } ukey_t;
static int cmp_ukey(const void *a, const void *b) {
  const ukey_t *x = (const ukey_t *)a, *y = (const ukey_t *)b;
  if (x->key < y->key) return -1;
  if (x->key > y->key) return 1;
  return (x->i > y->i) - (x->i < y->i);
}

int orc_fixup(const orc_problem *pr, const double *lam, int mode, unsigned char *x_out,
              double *P_out, double *R_out, int64_t *n_reset, int64_t *reset_list,
              int64_t reset_cap) {
  if (pr->M > MAXM) return -1;
  int M = pr->M, K = pr->K;
  int64_t N = pr->N;
  unsigned char *x = (unsigned char *)malloc((size_t)(N * M > 0 ? N * M : 1));
  double *G = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  double *R = (double *)malloc(sizeof(double) * (size_t)K);
  double g, P;
  orc_eval(pr, lam, x, R, &g, &P, G);
  unsigned char *viol = (unsigned char *)calloc((size_t)K, 1);
  int any = 0;
  for (int k = 0; k < K; ++k) { viol[k] = R[k] > pr->B[k]; any |= viol[k]; }
  /* per-user consumption row */
  double *v = (double *)malloc(sizeof(double) * (size_t)K);
  ukey_t *list = (ukey_t *)malloc(sizeof(ukey_t) * (size_t)(N > 0 ? N : 1));
  /* left[k]: exact consumption of violated knapsack k by the users not reset */
  xsum *left = (xsum *)calloc((size_t)K, sizeof(xsum));
  int64_t n = 0;
  for (int64_t i = 0; i < N && any; ++i) {
    int uses = 0;
    for (int k = 0; k < K; ++k) v[k] = 0.0;
    for (int j = 0; j < M; ++j) {
      int64_t r = i * M + j;
      if (!x[r]) continue;
      if (pr->b_format == 0) {
        for (int k = 0; k < K; ++k) {
          v[k] = v[k] + (double)pr->b[r * K + k];
          if (viol[k]) xsum_add(&left[k], (double)pr->b[r * K + k]);
        }
      } else {
        for (int64_t e = pr->rowptr[r]; e < pr->rowptr[r + 1]; ++e) {
          v[pr->col[e]] = v[pr->col[e]] + (double)pr->val[e];
          if (viol[pr->col[e]]) xsum_add(&left[pr->col[e]], (double)pr->val[e]);
        }
      }
    }
    for (int k = 0; k < K; ++k) uses |= viol[k] && v[k] > 0.0;
    if (mode == 1 || uses) { list[n].key = G[i]; list[n].i = i; ++n; }
  }
  qsort(list, (size_t)n, sizeof(ukey_t), cmp_ukey);
  int64_t reset = 0;
  for (int64_t t = 0; t < n; ++t) {
    int ok = 1;
    for (int k = 0; k < K; ++k) ok &= !viol[k] || xsum_cmp(&left[k], pr->B[k]) <= 0;
    if (ok) break;
    int64_t i = list[t].i;
    for (int j = 0; j < M; ++j) {
      int64_t r = i * M + j;
      if (!x[r]) continue;
      x[r] = 0;
      if (pr->b_format == 0) {
        for (int k = 0; k < K; ++k)
          if (viol[k]) xsum_add(&left[k], -(double)pr->b[r * K + k]);
      } else {
        for (int64_t e = pr->rowptr[r]; e < pr->rowptr[r + 1]; ++e)
          if (viol[pr->col[e]]) xsum_add(&left[pr->col[e]], -(double)pr->val[e]);
      }
    }
    if (reset_list && reset < reset_cap) reset_list[reset] = i;
    ++reset;
  }
  /* primal value and consumption of the projected solution, recomputed */
  nsum Ps = {0, 0};
  for (int k = 0; k < K; ++k) R[k] = 0.0;
  nsum *Rs = (nsum *)calloc((size_t)K, sizeof(nsum));
  for (int64_t i = 0; i < N; ++i) {
    double Pi = 0.0;
    for (int k = 0; k < K; ++k) v[k] = 0.0;
    for (int j = 0; j < M; ++j) {
      int64_t r = i * M + j;
      if (!x[r]) continue;
      Pi = Pi + (double)pr->p[r];
      if (pr->b_format == 0) {
        for (int k = 0; k < K; ++k) v[k] = v[k] + (double)pr->b[r * K + k];
      } else {
        for (int64_t e = pr->rowptr[r]; e < pr->rowptr[r + 1]; ++e)
          v[pr->col[e]] = v[pr->col[e]] + (double)pr->val[e];
      }
    }
    nadd(&Ps, Pi);
    for (int k = 0; k < K; ++k) nadd(&Rs[k], v[k]);
  }
  for (int k = 0; k < K; ++k) R_out[k] = nval(&Rs[k]);
  *P_out = nval(&Ps);
  *n_reset = reset;
  if (x_out) memcpy(x_out, x, (size_t)(N * M));
  free(Rs); free(x); free(G); free(R); free(viol); free(v); free(list); free(left);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 5 (Sec. 5.1): linear-time candidates for the special case       */
/* M = K, b_ijk = 0 for j != k, one top-Q constraint.  For user i emits at    */
/* most one (v1, v2) per k.  Reading: quick_select(a, n) is the n-th largest  */
/* value (0 when n exceeds K); ties compare with >= as printed; a zero        */
/* divisor b_ikk = 0 emits nothing.  Returns the number of pairs written.    */
/* ------------------------------------------------------------------------ */
static double nth_largest(const double *a, int n, int q) {
  if (q > n || q < 1) return 0.0;
  double tmp[MAXM];
  for (int t = 0; t < n; ++t) tmp[t] = a[t];
  for (int x1 = 1; x1 < n; ++x1) {
    double v = tmp[x1]; int y = x1 - 1;
    while (y >= 0 && tmp[y] < v) { tmp[y + 1] = tmp[y]; --y; }
    tmp[y + 1] = v;
  }
  return tmp[q - 1];
}

int orc_alg5_map_user(const orc_problem *pr, const double *lam, int64_t i, int Q,
                      int32_t *kk, double *v1, double *v2) {
  int K = pr->K;
  if (K > MAXM || pr->M != K) return -1;
  double adj[MAXM];
  for (int k = 0; k < K; ++k) {
    double bkk = b_at(pr, i * K + k, k);
    double prod = lam[k] * bkk;
    double a = (double)pr->p[i * K + k] - prod;
    adj[k] = a > 0.0 ? a : 0.0;
  }
  double qth = nth_largest(adj, K, Q), q1th = nth_largest(adj, K, Q + 1);
  int n = 0;
  for (int k = 0; k < K; ++k) {
    double pbar = adj[k] >= qth ? q1th : qth;
    double pk = (double)pr->p[i * K + k];
    double bkk = b_at(pr, i * K + k, k);
    if (pk > pbar && bkk > 0.0) {
      double num = pk - pbar;
      kk[n] = k; v1[n] = num / bkk; v2[n] = bkk; ++n;
    }
  }
  return n;
}

int orc_max_items(void) { return MAXM; }

/* Threads of the OpenMP loops over users (n >= 1); the results do not
   depend on it.  Returns the thread count in effect. */
int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* Cost-adjusted profits of users [u0,u1) into out[(i-u0)*M + j]. */
void orc_scores(const orc_problem *pr, const double *lam, int64_t u0, int64_t u1, double *out) {
  for (int64_t i = u0; i < u1; ++i) score_user(pr, lam, i, out + (i - u0) * pr->M);
}

/* Algorithm 1 on explicit values z[M] with the problem's local constraints. */
void orc_alg1(const orc_problem *pr, const double *z, unsigned char *x) {
  orc_sets s; sets_build(pr, &s);
  alg1(&s, z, x);
  sets_free(&s);
}
