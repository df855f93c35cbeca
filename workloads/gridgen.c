/*
 * Seeded random downward-closed grids for the batched workload (an input
 * generator, shared as input by the CPU oracle and the GPU library; it
 * evaluates nothing the method computes).
 *
 * A grid is a set of (level, odd index) multi-indices of one component, k <= 2
 * dimensions, level l_q >= 1 and odd 0 < i_q < 2^l_q per dimension.  Growth
 * starts at the root (1, ..., 1) and repeatedly adds a uniformly chosen
 * admissible point -- a point not in the grid whose parents (one per
 * dimension with l_q > 1: level l_q - 1, the odd index of (i_q -+ 1) / 2) are
 * all in the grid -- until the grid holds at least `target` points or no
 * admissible point is left.  Levels are capped at `lcap` per dimension.
 * Points are returned in the order they were added.  Random numbers come from
 * splitmix64 seeded with `seed`.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t sm64(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* open-addressing set of 64-bit keys (key 0 is never used: levels >= 1) */
typedef struct {
  uint64_t *slot;
  uint64_t mask;
} keyset;

static int ks_init(keyset *S, int64_t expect) {
  uint64_t cap = 1024;
  while (cap < (uint64_t)expect * 4) cap <<= 1;
  S->slot = (uint64_t *)calloc(cap, sizeof(uint64_t));
  S->mask = cap - 1;
  return S->slot ? 0 : -1;
}

static uint64_t ks_hash(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  return k;
}

static int ks_has(const keyset *S, uint64_t k) {
  for (uint64_t h = ks_hash(k) & S->mask;; h = (h + 1) & S->mask) {
    if (S->slot[h] == k) return 1;
    if (S->slot[h] == 0) return 0;
  }
}

static void ks_add(keyset *S, uint64_t k) {
  for (uint64_t h = ks_hash(k) & S->mask;; h = (h + 1) & S->mask) {
    if (S->slot[h] == k) return;
    if (S->slot[h] == 0) {
      S->slot[h] = k;
      return;
    }
  }
}

/* key of a point: per dimension 6 bits of level and 26 bits of index */
static uint64_t pkey(int k, const uint8_t *l, const uint32_t *i) {
  uint64_t key = 0;
  for (int q = 0; q < k; ++q) key = (key << 32) | ((uint64_t)l[q] << 26) | (uint64_t)i[q];
  return key;
}

static int parents_in(const keyset *G, int k, const uint8_t *l, const uint32_t *i) {
  for (int q = 0; q < k; ++q) {
    if (l[q] <= 1) continue;
    uint8_t pl[2];
    uint32_t pi[2];
    for (int r = 0; r < k; ++r) {
      pl[r] = l[r];
      pi[r] = i[r];
    }
    pl[q] = (uint8_t)(l[q] - 1);
    const uint32_t a = (i[q] - 1) / 2, b = (i[q] + 1) / 2;
    pi[q] = (a & 1u) ? a : b;
    if (!ks_has(G, pkey(k, pl, pi))) return 0;
  }
  return 1;
}

/* Returns the number of points written (<= cap), or -1 on a bad argument or
 * allocation failure.  lv, ix: cap x k (row-major). */
int64_t gg_closed_grid(int32_t k, int64_t target, int32_t lcap, uint64_t seed, uint8_t *lv, uint32_t *ix,
                       int64_t cap) {
  if (k < 1 || k > 2 || target < 1 || cap < 1 || lcap < 1 || lcap > 26 || !lv || !ix) return -1;
  if (target > cap) target = cap;
  keyset G, Cs;
  if (ks_init(&G, target + 16) || ks_init(&Cs, 4 * target + 64)) {
    free(G.slot);
    return -1;
  }
  int64_t ccap = 4 * target + 64, nc = 0;
  uint8_t *cl = (uint8_t *)malloc((size_t)ccap * 2);
  uint32_t *ci = (uint32_t *)malloc((size_t)ccap * 2 * sizeof(uint32_t));
  if (!cl || !ci) {
    free(G.slot);
    free(Cs.slot);
    free(cl);
    free(ci);
    return -1;
  }
  uint64_t s = seed;
  int64_t n = 0;
  /* the root */
  for (int q = 0; q < k; ++q) {
    cl[q] = 1;
    ci[q] = 1;
  }
  nc = 1;
  ks_add(&Cs, pkey(k, cl, ci));
  while (n < target && nc > 0) {
    const int64_t pick = (int64_t)(sm64(&s) % (uint64_t)nc);
    uint8_t l[2];
    uint32_t i[2];
    for (int q = 0; q < k; ++q) {
      l[q] = cl[pick * 2 + q];
      i[q] = ci[pick * 2 + q];
    }
    /* swap-remove the candidate, add the point */
    for (int q = 0; q < k; ++q) {
      cl[pick * 2 + q] = cl[(nc - 1) * 2 + q];
      ci[pick * 2 + q] = ci[(nc - 1) * 2 + q];
    }
    --nc;
    ks_add(&G, pkey(k, l, i));
    for (int q = 0; q < k; ++q) {
      lv[n * k + q] = l[q];
      ix[n * k + q] = i[q];
    }
    ++n;
    /* children that became admissible */
    for (int q = 0; q < k; ++q) {
      if (l[q] + 1 > lcap) continue;
      for (int side = -1; side <= 1; side += 2) {
        uint8_t chl[2];
        uint32_t chi[2];
        for (int r = 0; r < k; ++r) {
          chl[r] = l[r];
          chi[r] = i[r];
        }
        chl[q] = (uint8_t)(l[q] + 1);
        chi[q] = 2 * i[q] + (uint32_t)side;
        const uint64_t key = pkey(k, chl, chi);
        if (ks_has(&Cs, key) || ks_has(&G, key) || !parents_in(&G, k, chl, chi)) continue;
        if (nc == ccap) {
          ccap *= 2;
          uint8_t *ncl = (uint8_t *)realloc(cl, (size_t)ccap * 2);
          if (!ncl) goto oom;
          cl = ncl;
          uint32_t *nci = (uint32_t *)realloc(ci, (size_t)ccap * 2 * sizeof(uint32_t));
          if (!nci) goto oom;
          ci = nci;
        }
        for (int r = 0; r < k; ++r) {
          cl[nc * 2 + r] = chl[r];
          ci[nc * 2 + r] = chi[r];
        }
        ++nc;
        ks_add(&Cs, key);
      }
    }
  }
  free(G.slot);
  free(Cs.slot);
  free(cl);
  free(ci);
  return n;
oom:
  free(G.slot);
  free(Cs.slot);
  free(cl);
  free(ci);
  return -1;
}
