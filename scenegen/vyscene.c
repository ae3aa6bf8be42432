/*
 * Seeded synthetic city scene + LoD hierarchy builder (input generator).
 *
 * This file produces INPUT DATA only. It serves the FP64 oracle and the HIP
 * renderer alike and contains none of the rendering method's arithmetic
 * (no LoD predicate, projection, SH evaluation, binning, sorting or blending).
 *
 * Randomness: every draw is a counter-based SplitMix64 value (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014): the
 * 64-bit state for draw i of stream s is  key(seed, s) + i * GAMMA  and the
 * output is the SplitMix64 finaliser of that state. Results are therefore
 * independent of the thread count. Normals use the Box-Muller transform.
 *
 * Hierarchy: binary tree from recursive median split of the leaf means along
 * the longest axis of their bounding box; nodes numbered in breadth-first
 * order so that the children of a node are contiguous; each internal node is
 * the moment-matched merge of its two children (weights w = theta*sqrt(det
 * Sigma)); parent opacity 1 - prod(1 - theta_i); parent SH = weighted mean.
 * Node AABB = union(children AABBs, own 3-sigma box), the own box rounded
 * outward to fp32, so AABB(child) is contained in AABB(parent) exactly in fp32.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline uint64_t sm_key(uint64_t seed, uint64_t stream) {
  return sm_mix(seed * GAMMA + sm_mix(stream + 0x632BE59BD9B4E019ULL));
}
static inline double sm_uniform(uint64_t key, uint64_t i) {
  uint64_t x = sm_mix(key + (i + 1) * GAMMA);
  return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}
static inline double sm_normal(uint64_t key, uint64_t i) {
  double u1 = sm_uniform(key, 2 * i), u2 = sm_uniform(key, 2 * i + 1);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}

enum { ST_PLACE = 1, ST_SCALE = 2, ST_QUAT = 3, ST_OPAC = 4, ST_SH = 5 };

/* Draw the leaves.
 * buildings: n_b rows of (cx, cy, half_x, half_y, height).
 * Outputs (fp32): mean[n][3], log_scale[n][3], quat[n][4] (w,x,y,z),
 * logit[n], sh[n][16][3]. */
void vs_gen_leaves(uint64_t seed, int64_t n, double extent, double ground_frac,
                   int64_t n_b, const double* buildings,
                   double log_scale_mu, double log_scale_sigma,
                   double logit_sigma, double sh_dc_mu, double sh_sigma,
                   float* mean, float* log_scale, float* quat, float* logit, float* sh) {
  const uint64_t kp = sm_key(seed, ST_PLACE), ks = sm_key(seed, ST_SCALE),
                 kq = sm_key(seed, ST_QUAT), ko = sm_key(seed, ST_OPAC), kh = sm_key(seed, ST_SH);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double u[6];
    for (int k = 0; k < 6; ++k) u[k] = sm_uniform(kp, (uint64_t)i * 6 + k);
    double x, y, z;
    if (n_b == 0 || u[0] < ground_frac) {
      x = (u[1] - 0.5) * extent;
      y = (u[2] - 0.5) * extent;
      z = 0.0;
    } else {
      int64_t b = (int64_t)(u[1] * (double)n_b);
      if (b >= n_b) b = n_b - 1;
      const double* B = buildings + 5 * b;
      double cx = B[0], cy = B[1], hx = B[2], hy = B[3], h = B[4];
      double a_wx = 2.0 * hx * h, a_wy = 2.0 * hy * h, a_roof = 4.0 * hx * hy;
      double tot = 2.0 * a_wx + 2.0 * a_wy + a_roof;
      double f = u[2] * tot, s = u[3], t = u[4];
      if (f < a_wx) {                 /* wall at y = cy - hy */
        x = cx + (2 * s - 1) * hx; y = cy - hy; z = t * h;
      } else if (f < 2 * a_wx) {      /* wall at y = cy + hy */
        x = cx + (2 * s - 1) * hx; y = cy + hy; z = t * h;
      } else if (f < 2 * a_wx + a_wy) { /* wall at x = cx - hx */
        x = cx - hx; y = cy + (2 * s - 1) * hy; z = t * h;
      } else if (f < 2 * a_wx + 2 * a_wy) {
        x = cx + hx; y = cy + (2 * s - 1) * hy; z = t * h;
      } else {                        /* roof */
        x = cx + (2 * s - 1) * hx; y = cy + (2 * t - 1) * hy; z = h;
      }
    }
    mean[3 * i + 0] = (float)x; mean[3 * i + 1] = (float)y; mean[3 * i + 2] = (float)z;
    for (int k = 0; k < 3; ++k)
      log_scale[3 * i + k] = (float)(log_scale_mu + log_scale_sigma * sm_normal(ks, (uint64_t)i * 3 + k));
    double q[4], qn = 0.0;
    for (int k = 0; k < 4; ++k) { q[k] = sm_normal(kq, (uint64_t)i * 4 + k); qn += q[k] * q[k]; }
    qn = sqrt(qn);
    if (qn < 1e-12) { q[0] = 1; q[1] = q[2] = q[3] = 0; qn = 1; }
    for (int k = 0; k < 4; ++k) quat[4 * i + k] = (float)(q[k] / qn);
    logit[i] = (float)(logit_sigma * sm_normal(ko, (uint64_t)i));
    for (int k = 0; k < 48; ++k) {
      double v = sh_sigma * sm_normal(kh, (uint64_t)i * 48 + k);
      if (k < 3) v += sh_dc_mu;
      sh[48 * i + k] = (float)v;
    }
  }
}

/* ---------------- median-split tree structure ---------------- */

typedef struct { float key; int32_t idx; } kv_t;

static inline int kv_less(kv_t a, kv_t b) { return a.key < b.key || (a.key == b.key && a.idx < b.idx); }

/* Deterministic quickselect on (key, idx): afterwards a[k] is the k-th smallest
 * and a[0..k) <= a[k] <= a(k..n). Keys are made distinct by idx. */
static void kv_select(kv_t* a, int64_t n, int64_t k) {
  int64_t lo = 0, hi = n - 1;
  while (hi > lo) {
    int64_t mid = lo + (hi - lo) / 2;
    /* median of three into a[hi] as pivot */
    if (kv_less(a[mid], a[lo])) { kv_t t = a[mid]; a[mid] = a[lo]; a[lo] = t; }
    if (kv_less(a[hi], a[lo])) { kv_t t = a[hi]; a[hi] = a[lo]; a[lo] = t; }
    if (kv_less(a[mid], a[hi])) { kv_t t = a[mid]; a[mid] = a[hi]; a[hi] = t; }
    kv_t p = a[hi];
    int64_t s = lo;
    for (int64_t i = lo; i < hi; ++i)
      if (kv_less(a[i], p)) { kv_t t = a[i]; a[i] = a[s]; a[s] = t; ++s; }
    a[hi] = a[s]; a[s] = p;
    if (s == k) return;
    if (s < k) lo = s + 1; else hi = s - 1;
  }
}

/* Build the tree structure. perm[n_leaf] receives leaf ids grouped by segment.
 * Outputs per node (n_node = 2*n_leaf-1): parent, first_child (-1 leaf),
 * child_count (0 or 2), leaf_of (-1 internal). level_start[depth+2] gets the
 * first node id of every BFS level (returns the number of levels). */
int vs_build_tree(int64_t n_leaf, const float* mean, int32_t* parent, int32_t* first_child,
                  int32_t* child_count, int32_t* leaf_of, int64_t* level_start, int max_levels) {
  int64_t n_node = 2 * n_leaf - 1;
  int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * n_leaf);
  kv_t* buf = (kv_t*)malloc(sizeof(kv_t) * n_leaf);
  int64_t* seg = (int64_t*)malloc(sizeof(int64_t) * 2 * n_leaf);   /* lo,hi of current level */
  int64_t* nseg = (int64_t*)malloc(sizeof(int64_t) * 2 * n_leaf);
  int64_t* rank = (int64_t*)malloc(sizeof(int64_t) * (n_leaf + 1));
  if (!perm || !buf || !seg || !nseg || !rank) return -1;
  for (int64_t i = 0; i < n_leaf; ++i) perm[i] = (int32_t)i;
  int64_t cnt = 1, base = 0;
  seg[0] = 0; seg[1] = n_leaf;
  parent[0] = -1;
  int lev = 0;
  while (cnt > 0) {
    if (lev + 1 >= max_levels) return -2;
    level_start[lev] = base;
    /* child base ids: exclusive prefix of 2*(internal) */
    rank[0] = 0;
    for (int64_t j = 0; j < cnt; ++j) rank[j + 1] = rank[j] + ((seg[2 * j + 1] - seg[2 * j]) > 1 ? 1 : 0);
    int64_t next_base = base + cnt;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < cnt; ++j) {
      int64_t lo = seg[2 * j], hi = seg[2 * j + 1], sz = hi - lo, id = base + j;
      if (sz == 1) {
        first_child[id] = -1; child_count[id] = 0; leaf_of[id] = perm[lo];
        continue;
      }
      double bl[3] = {INFINITY, INFINITY, INFINITY}, bh[3] = {-INFINITY, -INFINITY, -INFINITY};
      for (int64_t i = lo; i < hi; ++i)
        for (int k = 0; k < 3; ++k) {
          double v = mean[3 * (int64_t)perm[i] + k];
          if (v < bl[k]) bl[k] = v;
          if (v > bh[k]) bh[k] = v;
        }
      int ax = 0;
      for (int k = 1; k < 3; ++k) if (bh[k] - bl[k] > bh[ax] - bl[ax]) ax = k;
      for (int64_t i = lo; i < hi; ++i) { buf[i].key = mean[3 * (int64_t)perm[i] + ax]; buf[i].idx = perm[i]; }
      int64_t half = sz / 2;
      kv_select(buf + lo, sz, half);
      for (int64_t i = lo; i < hi; ++i) perm[i] = buf[i].idx;
      int64_t c = next_base + 2 * rank[j];
      first_child[id] = (int32_t)c; child_count[id] = 2; leaf_of[id] = -1;
      parent[c] = (int32_t)id; parent[c + 1] = (int32_t)id;
      nseg[4 * rank[j] + 0] = lo; nseg[4 * rank[j] + 1] = lo + half;
      nseg[4 * rank[j] + 2] = lo + half; nseg[4 * rank[j] + 3] = hi;
    }
    int64_t ncnt = 2 * rank[cnt];
    base = next_base;
    int64_t* t = seg; seg = nseg; nseg = t;
    cnt = ncnt;
    ++lev;
  }
  level_start[lev] = base;
  free(perm); free(buf); free(seg); free(nseg); free(rank);
  if (base != n_node) return -3;
  return lev;
}

/* ---------------- per-node attributes ---------------- */

static void quat_to_rot(const double q[4], double R[9]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* Rotation matrix (columns = axes) to unit quaternion (w,x,y,z), Shepperd's method. */
static void rot_to_quat(const double R[9], double q[4]) {
  double tr = R[0] + R[4] + R[8];
  if (tr > 0) {
    double s = sqrt(tr + 1.0) * 2;
    q[0] = 0.25 * s; q[1] = (R[7] - R[5]) / s; q[2] = (R[2] - R[6]) / s; q[3] = (R[3] - R[1]) / s;
  } else if (R[0] > R[4] && R[0] > R[8]) {
    double s = sqrt(1.0 + R[0] - R[4] - R[8]) * 2;
    q[0] = (R[7] - R[5]) / s; q[1] = 0.25 * s; q[2] = (R[1] + R[3]) / s; q[3] = (R[2] + R[6]) / s;
  } else if (R[4] > R[8]) {
    double s = sqrt(1.0 + R[4] - R[0] - R[8]) * 2;
    q[0] = (R[2] - R[6]) / s; q[1] = (R[1] + R[3]) / s; q[2] = 0.25 * s; q[3] = (R[5] + R[7]) / s;
  } else {
    double s = sqrt(1.0 + R[8] - R[0] - R[4]) * 2;
    q[0] = (R[3] - R[1]) / s; q[1] = (R[2] + R[6]) / s; q[2] = (R[5] + R[7]) / s; q[3] = 0.25 * s;
  }
  double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) q[k] /= n;
}

/* Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix (row-major A).
 * Eigenvalues in w, eigenvectors as the columns of V. */
static void jacobi3(const double A_in[9], double w[3], double V[9]) {
  double A[9];
  memcpy(A, A_in, sizeof(A));
  for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = fabs(A[1]) + fabs(A[2]) + fabs(A[5]);
    double scale = fabs(A[0]) + fabs(A[4]) + fabs(A[8]);
    if (off <= 1e-300 || off < 1e-17 * scale) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        double apq = A[3 * p + q];
        if (fabs(apq) < 1e-300) continue;
        double app = A[3 * p + p], aqq = A[3 * q + q];
        double theta = (aqq - app) / (2 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) { /* A = J^T A J on columns p,q */
          double akp = A[3 * k + p], akq = A[3 * k + q];
          A[3 * k + p] = c * akp - s * akq;
          A[3 * k + q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
          double apk = A[3 * p + k], aqk = A[3 * q + k];
          A[3 * p + k] = c * apk - s * aqk;
          A[3 * q + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          double vkp = V[3 * k + p], vkq = V[3 * k + q];
          V[3 * k + p] = c * vkp - s * vkq;
          V[3 * k + q] = s * vkp + c * vkq;
        }
      }
  }
  w[0] = A[0]; w[1] = A[4]; w[2] = A[8];
}

static inline float round_down_f32(double v) {
  float f = (float)v;
  if ((double)f > v) f = nextafterf(f, -INFINITY);
  return f;
}
static inline float round_up_f32(double v) {
  float f = (float)v;
  if ((double)f < v) f = nextafterf(f, INFINITY);
  return f;
}

/* Fill every node's attributes bottom-up (levels from deepest to root).
 * Leaf attributes are read from the leaf arrays via leaf_of; internal nodes are
 * moment-matched merges of their two children. Outputs fp32 per node. */
int vs_fill_nodes(int64_t n_leaf, int nlev, const int64_t* level_start,
                  const int32_t* first_child, const int32_t* leaf_of,
                  const float* l_mean, const float* l_log_scale, const float* l_quat,
                  const float* l_logit, const float* l_sh,
                  float* mean, float* log_scale, float* quat, float* logit, float* sh,
                  float* aabb_lo, float* aabb_hi, double logit_clamp) {
  int64_t n_node = 2 * n_leaf - 1;
  double* tmp = (double*)malloc(sizeof(double) * 11 * n_node); /* mu3, cov6, w, log(1-theta) */
  if (!tmp) return -1;
  for (int lev = nlev - 1; lev >= 0; --lev) {
    int64_t a = level_start[lev], b = level_start[lev + 1];
#pragma omp parallel for schedule(static)
    for (int64_t id = a; id < b; ++id) {
      double* T = tmp + 11 * id;
      double mu[3], C[9], theta, lq;
      if (first_child[id] < 0) {
        int64_t L = leaf_of[id];
        double q[4], qn = 0, R[9], s[3];
        for (int k = 0; k < 4; ++k) { q[k] = l_quat[4 * L + k]; qn += q[k] * q[k]; }
        qn = sqrt(qn);
        for (int k = 0; k < 4; ++k) q[k] /= qn;
        quat_to_rot(q, R);
        for (int k = 0; k < 3; ++k) { mu[k] = l_mean[3 * L + k]; s[k] = exp((double)l_log_scale[3 * L + k]); }
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) {
            double v = 0;
            for (int k = 0; k < 3; ++k) v += R[3 * i + k] * s[k] * s[k] * R[3 * j + k];
            C[3 * i + j] = v;
          }
        double lg = l_logit[L];
        theta = 1.0 / (1.0 + exp(-lg));
        lq = -log1p(exp(lg)); /* log(1 - theta) */
        for (int k = 0; k < 3; ++k) { mean[3 * id + k] = l_mean[3 * L + k]; log_scale[3 * id + k] = l_log_scale[3 * L + k]; }
        for (int k = 0; k < 4; ++k) quat[4 * id + k] = l_quat[4 * L + k];
        logit[id] = l_logit[L];
        memcpy(sh + 48 * id, l_sh + 48 * L, 48 * sizeof(float));
        T[9] = theta * s[0] * s[1] * s[2];
        for (int k = 0; k < 3; ++k) {
          double hw = 3.0 * sqrt(C[4 * k]);
          aabb_lo[3 * id + k] = round_down_f32(mu[k] - hw);
          aabb_hi[3 * id + k] = round_up_f32(mu[k] + hw);
        }
      } else {
        int64_t c0 = first_child[id], c1 = c0 + 1;
        const double *A = tmp + 11 * c0, *B = tmp + 11 * c1;
        double wa = A[9], wb = B[9], w = wa + wb;
        if (!(w > 0)) { wa = wb = 0.5; w = 1.0; }
        for (int k = 0; k < 3; ++k) mu[k] = (wa * A[k] + wb * B[k]) / w;
        double da[3], db[3];
        for (int k = 0; k < 3; ++k) { da[k] = A[k] - mu[k]; db[k] = B[k] - mu[k]; }
        int idx6[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            C[3 * i + j] = (wa * (A[3 + idx6[3 * i + j]] + da[i] * da[j]) +
                            wb * (B[3 + idx6[3 * i + j]] + db[i] * db[j])) / w;
        lq = A[10] + B[10];
        theta = -expm1(lq);
        double lgt = log(theta) - lq;
        if (lgt > logit_clamp) lgt = logit_clamp;
        if (lgt < -logit_clamp) lgt = -logit_clamp;
        double ev[3], V[9];
        jacobi3(C, ev, V);
        /* make V a proper rotation */
        double det = V[0] * (V[4] * V[8] - V[5] * V[7]) - V[1] * (V[3] * V[8] - V[5] * V[6]) +
                     V[2] * (V[3] * V[7] - V[4] * V[6]);
        if (det < 0) { V[2] = -V[2]; V[5] = -V[5]; V[8] = -V[8]; }
        double q[4];
        rot_to_quat(V, q);
        double sd = 1.0;
        for (int k = 0; k < 3; ++k) {
          double e = ev[k] > 1e-12 ? ev[k] : 1e-12;
          log_scale[3 * id + k] = (float)(0.5 * log(e));
          sd *= sqrt(e);
        }
        for (int k = 0; k < 4; ++k) quat[4 * id + k] = (float)q[k];
        for (int k = 0; k < 3; ++k) mean[3 * id + k] = (float)mu[k];
        logit[id] = (float)lgt;
        for (int k = 0; k < 48; ++k)
          sh[48 * id + k] = (float)((wa * sh[48 * c0 + k] + wb * sh[48 * c1 + k]) / w);
        T[9] = theta * sd;
        for (int k = 0; k < 3; ++k) {
          double hw = 3.0 * sqrt(C[4 * k]);
          float lo = round_down_f32(mu[k] - hw), hi = round_up_f32(mu[k] + hw);
          float l0 = aabb_lo[3 * c0 + k], l1 = aabb_lo[3 * c1 + k];
          float h0 = aabb_hi[3 * c0 + k], h1 = aabb_hi[3 * c1 + k];
          if (l0 < lo) lo = l0;
          if (l1 < lo) lo = l1;
          if (h0 > hi) hi = h0;
          if (h1 > hi) hi = h1;
          aabb_lo[3 * id + k] = lo; aabb_hi[3 * id + k] = hi;
        }
      }
      for (int k = 0; k < 3; ++k) T[k] = mu[k];
      T[3] = C[0]; T[4] = C[1]; T[5] = C[2]; T[6] = C[4]; T[7] = C[5]; T[8] = C[8];
      T[10] = lq;
    }
  }
  free(tmp);
  return 0;
}

int vs_num_threads(void) { return omp_get_max_threads(); }
