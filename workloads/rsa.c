/*
 * rsa.c -- random sequential adsorption filter for synthetic initial states.
 *
 * Candidates are visited in order; a candidate is accepted when no accepted
 * point lies closer than dmin (minimum image along periodic dimensions).
 * Stops after `target` acceptances.  Pure geometry: no part of the
 * integration method lives here.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static uint64_t cell_hash(int64_t cx, int64_t cy, int64_t cz) {
  uint64_t h = (uint64_t)cx * 0x9E3779B97F4A7C15ull;
  h ^= (uint64_t)cy * 0xC2B2AE3D27D4EB4Full + (h << 6) + (h >> 2);
  h ^= (uint64_t)cz * 0x165667B19E3779F9ull + (h << 6) + (h >> 2);
  h ^= h >> 31;
  return h;
}

static int64_t cell_of(double v, double lo, double cs, int64_t nc, int per) {
  int64_t c = (int64_t)floor((v - lo) / cs);
  if (per) {
    c %= nc;
    if (c < 0) c += nc;
  }
  return c;
}

/* Returns the number of accepted points written to out (3 doubles each),
 * or -1 on allocation failure. */
int64_t rsa_filter(const double* cand, int64_t m, double dmin, const double* lo, const double* hi,
                   const int* periodic, int64_t target, double* out) {
  uint64_t nb = 1;
  while (nb < 2 * (uint64_t)(target > 0 ? target : 1)) nb <<= 1;
  int64_t* head = (int64_t*)malloc(sizeof(int64_t) * nb);
  int64_t* next = (int64_t*)malloc(sizeof(int64_t) * (size_t)(target > 0 ? target : 1));
  if (!head || !next) {
    free(head);
    free(next);
    return -1;
  }
  for (uint64_t b = 0; b < nb; ++b) head[b] = -1;
  double cs[3], L[3];
  int64_t nc[3];
  for (int k = 0; k < 3; ++k) {
    L[k] = hi[k] - lo[k];
    if (periodic[k]) {
      nc[k] = (int64_t)floor(L[k] / dmin);
      if (nc[k] < 1) nc[k] = 1;
      cs[k] = L[k] / (double)nc[k];
    } else {
      nc[k] = 0;
      cs[k] = dmin;
    }
  }
  const double d2min = dmin * dmin;
  int64_t n = 0;
  for (int64_t t = 0; t < m && n < target; ++t) {
    const double* q = &cand[3 * t];
    int64_t c[3];
    for (int k = 0; k < 3; ++k) c[k] = cell_of(q[k], lo[k], cs[k], nc[k], periodic[k]);
    int ok = 1;
    for (int dx = -1; dx <= 1 && ok; ++dx)
      for (int dy = -1; dy <= 1 && ok; ++dy)
        for (int dz = -1; dz <= 1 && ok; ++dz) {
          int64_t cc[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
          for (int k = 0; k < 3; ++k)
            if (periodic[k]) cc[k] = ((cc[k] % nc[k]) + nc[k]) % nc[k];
          const uint64_t b = cell_hash(cc[0], cc[1], cc[2]) & (nb - 1);
          for (int64_t j = head[b]; j >= 0; j = next[j]) {
            double d[3];
            for (int k = 0; k < 3; ++k) {
              d[k] = q[k] - out[3 * j + k];
              if (periodic[k]) d[k] -= L[k] * nearbyint(d[k] / L[k]);
            }
            if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < d2min) {
              ok = 0;
              break;
            }
          }
        }
    if (!ok) continue;
    for (int k = 0; k < 3; ++k) out[3 * n + k] = q[k];
    const uint64_t b = cell_hash(c[0], c[1], c[2]) & (nb - 1);
    next[n] = head[b];
    head[b] = n;
    ++n;
  }
  free(head);
  free(next);
  return n;
}
