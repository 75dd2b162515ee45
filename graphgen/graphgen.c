/*
 * graphgen.c -- seeded synthetic graph inputs and CSR/CSC assembly.
 *
 * This module produces the *inputs* that both the CPU oracle and the GPU
 * library consume.  It holds none of the vertex-centric method's arithmetic:
 * no compute, no combine, no superstep.  Everything is deterministic for a
 * given seed and independent of the number of OpenMP threads.
 *
 * Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014) used as a
 * counter-based generator: draw k of a stream with base b is
 * mix64(b + (k+1) * 0x9E3779B97F4A7C15).  A stream therefore can be split
 * across threads at any index without changing a single value.
 *
 * R-MAT follows Chakrabarti, Zhan and Faloutsos (SDM 2004): each edge picks
 * one quadrant per level with probabilities (a, b, c, d); no noise, no vertex
 * permutation.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GG_GAMMA 0x9E3779B97F4A7C15ull

static inline uint64_t gg_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Draw number k (0-based) of the stream whose base is b. */
static inline uint64_t gg_draw(uint64_t b, uint64_t k) { return gg_mix64(b + (k + 1) * GG_GAMMA); }

/* 53-bit uniform double in [0, 1). */
static inline double gg_unit(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

/* Stream base for a (seed, purpose) pair. */
static inline uint64_t gg_base(uint64_t seed, uint64_t purpose) {
  return gg_mix64(seed * GG_GAMMA ^ gg_mix64(purpose + 0x632BE59BD9B4E019ull));
}

uint64_t gg_splitmix_draw(uint64_t seed, uint64_t purpose, uint64_t k) {
  return gg_draw(gg_base(seed, purpose), k);
}

/* ------------------------------------------------------------------------ */
/* R-MAT edge list: m edges over 2^scale ids.  Edge i uses draws
 * [i*scale, (i+1)*scale) of stream (seed, purpose=1).  Level l decides bit
 * (scale-1-l) of the source and destination ids. */
void gg_rmat_edges(int scale, uint64_t m, double a, double b, double c, uint64_t seed,
                   uint32_t* src, uint32_t* dst) {
  const uint64_t base = gg_base(seed, 1);
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)m; ++i) {
    uint32_t s = 0, d = 0;
    uint64_t k = (uint64_t)i * (uint64_t)scale;
    for (int l = 0; l < scale; ++l) {
      double r = gg_unit(gg_draw(base, k + (uint64_t)l));
      uint32_t bit = 1u << (scale - 1 - l);
      if (r < a) {
      } else if (r < ab) {
        d |= bit;
      } else if (r < abc) {
        s |= bit;
      } else {
        s |= bit;
        d |= bit;
      }
    }
    src[i] = s;
    dst[i] = d;
  }
}

/* R-MAT restricted to ids < n (n <= 2^scale): draws are taken in order and
 * kept while both ends are < n, until `want` edges are kept.  Returns the
 * number of draws consumed.  Single-threaded (small graphs). */
uint64_t gg_rmat_edges_bounded(int scale, uint32_t n, uint64_t want, double a, double b, double c,
                               uint64_t seed, uint32_t* src, uint32_t* dst) {
  const uint64_t base = gg_base(seed, 1);
  const double ab = a + b, abc = a + b + c;
  uint64_t kept = 0, drawn = 0;
  while (kept < want) {
    uint32_t s = 0, d = 0;
    uint64_t k = drawn * (uint64_t)scale;
    for (int l = 0; l < scale; ++l) {
      double r = gg_unit(gg_draw(base, k + (uint64_t)l));
      uint32_t bit = 1u << (scale - 1 - l);
      if (r < a) {
      } else if (r < ab) {
        d |= bit;
      } else if (r < abc) {
        s |= bit;
      } else {
        s |= bit;
        d |= bit;
      }
    }
    ++drawn;
    if (s < n && d < n) {
      src[kept] = s;
      dst[kept] = d;
      ++kept;
    }
  }
  return drawn;
}

/* ------------------------------------------------------------------------ */
/* In-place sort of a small int32 array (insertion sort below 32, else an
 * iterative introsort-free quicksort with median-of-three). */
static void gg_sort_i32(int32_t* x, int64_t n) {
  while (n > 32) {
    int32_t p0 = x[0], p1 = x[n / 2], p2 = x[n - 1];
    int32_t p = p0 < p1 ? (p1 < p2 ? p1 : (p0 < p2 ? p2 : p0)) : (p0 < p2 ? p0 : (p1 < p2 ? p2 : p1));
    int64_t i = 0, j = n - 1;
    for (;;) {
      while (x[i] < p) ++i;
      while (x[j] > p) --j;
      if (i >= j) break;
      int32_t t = x[i];
      x[i] = x[j];
      x[j] = t;
      ++i;
      --j;
    }
    /* recurse into the smaller half, loop on the larger */
    int64_t left = j + 1;
    if (left <= 0 || left >= n) break; /* cannot happen with a median-of-three pivot */
    if (left < n - left) {
      gg_sort_i32(x, left);
      x += left;
      n -= left;
    } else {
      gg_sort_i32(x + left, n - left);
      n = left;
    }
  }
  for (int64_t i = 1; i < n; ++i) {
    int32_t v = x[i];
    int64_t j = i - 1;
    while (j >= 0 && x[j] > v) {
      x[j + 1] = x[j];
      --j;
    }
    x[j + 1] = v;
  }
}

/* Count phase of CSR assembly.  deg must be zeroed, length n.
 * flags: bit0 symmetrise, bit1 keep self-loops. */
static void gg_count(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst, int flags,
                     uint64_t* deg) {
  const int sym = flags & 1, keep_loops = flags & 2;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)m; ++i) {
    uint32_t s = src[i], d = dst[i];
    if (s >= n || d >= n) continue;
    if (s == d && !keep_loops) continue;
    __atomic_fetch_add(&deg[s], 1, __ATOMIC_RELAXED);
    if (sym && s != d) __atomic_fetch_add(&deg[d], 1, __ATOMIC_RELAXED);
  }
}

/*
 * Assemble a CSR (out-adjacency) from an edge list.
 *   flags bit0: symmetrise (add the reverse of every edge)
 *   flags bit1: keep self-loops
 *   flags bit2: keep duplicate edges
 * Two calls: with adj == NULL it only fills off[0..n] (capacity before
 * dedup) and returns that capacity; with adj != NULL (capacity entries,
 * off from the first call) it fills, sorts each list, removes duplicates
 * unless asked not to, compacts, rewrites off and returns the final edge
 * count.  Edges with an endpoint >= n are ignored.
 */
uint64_t gg_build_csr(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst, int flags,
                      uint64_t* off, int32_t* adj) {
  const int sym = flags & 1, keep_loops = flags & 2, keep_dups = flags & 4;
  if (adj == NULL) {
    uint64_t* deg = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
    gg_count(n, m, src, dst, flags, deg);
    uint64_t acc = 0;
    for (uint32_t v = 0; v < n; ++v) {
      off[v] = acc;
      acc += deg[v];
    }
    off[n] = acc;
    free(deg);
    return acc;
  }
  uint64_t* cur = (uint64_t*)malloc(((size_t)n + 1) * sizeof(uint64_t));
  memcpy(cur, off, ((size_t)n + 1) * sizeof(uint64_t));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)m; ++i) {
    uint32_t s = src[i], d = dst[i];
    if (s >= n || d >= n) continue;
    if (s == d && !keep_loops) continue;
    uint64_t p = __atomic_fetch_add(&cur[s], 1, __ATOMIC_RELAXED);
    adj[p] = (int32_t)d;
    if (sym && s != d) {
      uint64_t q = __atomic_fetch_add(&cur[d], 1, __ATOMIC_RELAXED);
      adj[q] = (int32_t)s;
    }
  }
  /* sort and dedup each list in place; cur[v] becomes the kept length */
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t v = 0; v < (int64_t)n; ++v) {
    int32_t* a = adj + off[v];
    int64_t len = (int64_t)(off[v + 1] - off[v]);
    gg_sort_i32(a, len);
    int64_t k = len;
    if (!keep_dups && len > 1) {
      k = 1;
      for (int64_t j = 1; j < len; ++j)
        if (a[j] != a[k - 1]) a[k++] = a[j];
    }
    cur[v] = (uint64_t)k;
  }
  /* compact */
  uint64_t acc = 0;
  for (uint32_t v = 0; v < n; ++v) {
    uint64_t len = cur[v], from = off[v];
    off[v] = acc;
    if (from != acc) memmove(adj + acc, adj + from, len * sizeof(int32_t));
    acc += len;
  }
  off[n] = acc;
  free(cur);
  return acc;
}

/* Transpose a CSR into a CSC (in-adjacency): toff must hold n+1 entries,
 * tadj off[n] entries.  Each in-list is sorted ascending. */
void gg_transpose(uint32_t n, const uint64_t* off, const int32_t* adj, uint64_t* toff, int32_t* tadj) {
  const uint64_t m = off[n];
  uint64_t* deg = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < (int64_t)m; ++e) __atomic_fetch_add(&deg[adj[e]], 1, __ATOMIC_RELAXED);
  uint64_t acc = 0;
  for (uint32_t v = 0; v < n; ++v) {
    toff[v] = acc;
    acc += deg[v];
  }
  toff[n] = acc;
  memcpy(deg, toff, (size_t)n * sizeof(uint64_t));
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t u = 0; u < (int64_t)n; ++u)
    for (uint64_t e = off[u]; e < off[u + 1]; ++e) {
      uint64_t p = __atomic_fetch_add(&deg[adj[e]], 1, __ATOMIC_RELAXED);
      tadj[p] = (int32_t)u;
    }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t v = 0; v < (int64_t)n; ++v) gg_sort_i32(tadj + toff[v], (int64_t)(toff[v + 1] - toff[v]));
  free(deg);
}

/* Symmetrised form of a directed graph given as CSR + CSC with every list
 * sorted ascending and free of duplicates: vertex v's list is the sorted
 * union of its out- and in-list, without duplicates and without v itself.
 * (The same graph as drawing the edge list again and adding every edge
 * reversed, then dropping self-loops and duplicates.)  Two calls: with
 * sadj == NULL it fills soff[0..n] and returns the edge count; then with
 * sadj (that many entries) it fills the lists. */
static uint64_t gg_merge_len(const int32_t* a, uint64_t na, const int32_t* b, uint64_t nb, int32_t self,
                             int32_t* out) {
  uint64_t i = 0, j = 0, k = 0;
  while (i < na || j < nb) {
    int32_t x;
    if (j >= nb || (i < na && a[i] < b[j])) x = a[i++];
    else if (i >= na || b[j] < a[i]) x = b[j++];
    else {
      x = a[i++];
      ++j;
    }
    if (x == self) continue;
    if (out) out[k] = x;
    ++k;
  }
  return k;
}

uint64_t gg_symmetrise(uint32_t n, const uint64_t* off, const int32_t* adj, const uint64_t* toff, const int32_t* tadj,
                       uint64_t* soff, int32_t* sadj) {
  if (sadj == NULL) {
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < (int64_t)n; ++v)
      soff[v + 1] = gg_merge_len(adj + off[v], off[v + 1] - off[v], tadj + toff[v], toff[v + 1] - toff[v],
                                 (int32_t)v, NULL);
    soff[0] = 0;
    for (uint32_t v = 0; v < n; ++v) soff[v + 1] += soff[v];
    return soff[n];
  }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < (int64_t)n; ++v)
    gg_merge_len(adj + off[v], off[v + 1] - off[v], tadj + toff[v], toff[v + 1] - toff[v], (int32_t)v, sadj + soff[v]);
  return soff[n];
}

/* Per-edge weights of a CSR, symmetric in (u, v): w = lo + H(seed, min, max) % (hi-lo+1). */
void gg_edge_weights(uint32_t n, const uint64_t* off, const int32_t* adj, uint64_t seed, uint32_t lo,
                     uint32_t hi, uint32_t* w) {
  const uint64_t base = gg_base(seed, 7);
  const uint64_t span = (uint64_t)hi - lo + 1;
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t u = 0; u < (int64_t)n; ++u)
    for (uint64_t e = off[u]; e < off[u + 1]; ++e) {
      uint64_t v = (uint64_t)(uint32_t)adj[e];
      uint64_t x = (uint64_t)u < v ? (uint64_t)u : v, y = (uint64_t)u < v ? v : (uint64_t)u;
      uint64_t h = gg_mix64(base ^ gg_mix64((x << 32) | y));
      w[e] = lo + (uint32_t)(h % span);
    }
}

/* ------------------------------------------------------------------------ */
/* 2-D grid, 4-neighbour, row-major ids r*width+c; emits each undirected edge
 * once (right and down neighbours).  Returns the count (2*w*(w-1) for a
 * square grid).  src/dst must hold that many entries. */
uint64_t gg_grid_edges(uint32_t width, uint32_t height, uint32_t* src, uint32_t* dst) {
  uint64_t k = 0;
  for (uint32_t r = 0; r < height; ++r)
    for (uint32_t c = 0; c < width; ++c) {
      uint32_t v = r * width + c;
      if (c + 1 < width) {
        src[k] = v;
        dst[k] = v + 1;
        ++k;
      }
      if (r + 1 < height) {
        src[k] = v;
        dst[k] = v + width;
        ++k;
      }
    }
  return k;
}

typedef struct {
  uint64_t* keys;
  uint64_t cap;
} gg_set;

static int gg_set_insert(gg_set* s, uint64_t key) { /* key != 0; returns 1 if new */
  uint64_t h = gg_mix64(key) & (s->cap - 1);
  for (;;) {
    if (s->keys[h] == 0) {
      s->keys[h] = key;
      return 1;
    }
    if (s->keys[h] == key) return 0;
    h = (h + 1) & (s->cap - 1);
  }
}

/* `count` distinct long-range shortcut pairs on a width x height grid:
 * endpoints uniform, u != v, not grid-adjacent, no pair drawn twice
 * (unordered).  Stream (seed, purpose=3), draws taken in order. */
void gg_grid_shortcuts(uint32_t width, uint32_t height, uint64_t count, uint64_t seed, uint32_t* src,
                       uint32_t* dst) {
  const uint64_t base = gg_base(seed, 3);
  const uint64_t n = (uint64_t)width * height;
  gg_set set;
  set.cap = 1;
  while (set.cap < 4 * count + 16) set.cap <<= 1;
  set.keys = (uint64_t*)calloc(set.cap, sizeof(uint64_t));
  uint64_t kept = 0, k = 0;
  while (kept < count) {
    uint64_t u = gg_draw(base, k++) % n, v = gg_draw(base, k++) % n;
    if (u == v) continue;
    uint64_t ur = u / width, uc = u % width, vr = v / width, vc = v % width;
    uint64_t dr = ur > vr ? ur - vr : vr - ur, dc = uc > vc ? uc - vc : vc - uc;
    if (dr + dc == 1) continue;
    uint64_t x = u < v ? u : v, y = u < v ? v : u;
    if (!gg_set_insert(&set, ((x << 32) | y) + 1)) continue;
    src[kept] = (uint32_t)u;
    dst[kept] = (uint32_t)v;
    ++kept;
  }
  free(set.keys);
}

/* `count` distinct ids in [0, n) drawn uniformly among those with
 * eligible[v] != 0, in draw order.  Stream (seed, purpose=5). */
void gg_pick_sources(uint32_t n, const uint8_t* eligible, uint64_t count, uint64_t seed, uint32_t* out) {
  const uint64_t base = gg_base(seed, 5);
  gg_set set;
  set.cap = 1;
  while (set.cap < 4 * count + 16) set.cap <<= 1;
  set.keys = (uint64_t*)calloc(set.cap, sizeof(uint64_t));
  uint64_t kept = 0, k = 0;
  while (kept < count) {
    uint32_t v = (uint32_t)(gg_draw(base, k++) % n);
    if (!eligible[v]) continue;
    if (!gg_set_insert(&set, (uint64_t)v + 1)) continue;
    out[kept++] = v;
  }
  free(set.keys);
}

int gg_max_threads(void) { return omp_get_max_threads(); }
