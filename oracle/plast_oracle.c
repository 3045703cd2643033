/*
 * Plain C oracle for the PLAST-P bank-versus-bank hot path -- TEST INFRASTRUCTURE.
 *
 * Scalar, unblocked loops that state what the GPU library computes; used by the
 * tests on inputs too large for the numpy oracle and timed as the CPU baseline.
 * It shares no code, header, table or constant with the GPU library.  The
 * substitution matrix is passed in by the caller (the Python oracle's
 * transcription); the subset-seed classes are defined here.
 *
 * Paper: Nguyen & Lavenier, INRIA RR-6513 (2008).
 *   - seed key and index: Sec. 3.3.1 (subset-seed table, look-up table plus
 *     occurrence lists);
 *   - one-hit ungapped extension of every same-key pair: Sec. 3.2 generic
 *     algorithm and Sec. 3.3.3, score composition from the GPU kernel of
 *     Annex 4 (best rightward prefix, then best leftward prefix added to it);
 *   - work distribution: Sec. 5.1, threads take seeds one at a time from a
 *     shared counter;
 *   - small gapped filter: Sec. 3.3.4 (stage 3.1) and Sec. 5.2.2 (one
 *     extension on each side of the seed), banded affine-gap DP.
 *
 * Bank storage: codes[] holds, for sequence i, residues 0..19 at
 * [seq_start[i], seq_start[i+1] - pad); everything else is padding and is never
 * read here (scans are clipped at sequence ends).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NKEYS 8800
#define ORC_W 4

static const char ORC_ALPHA[] = "ACDEFGHIKLMNPQRSTVWY";
/* position-2 classes (2) and position-3 classes (11) of the subset seed */
static const char* ORC_POS2[2] = {"CFYWMLIV", "GPATSNHQEDRK"};
static const char* ORC_POS3[11] = {"A", "C", "FYW", "G", "IV", "ML", "NH", "P", "QED", "RK", "TS"};

static int orc_letter(char c) {
  for (int i = 0; i < 20; ++i)
    if (ORC_ALPHA[i] == c) return i;
  return -1;
}

static void orc_classes(int c2[20], int c3[20]) {
  for (int k = 0; k < 2; ++k)
    for (const char* p = ORC_POS2[k]; *p; ++p) c2[orc_letter(*p)] = k;
  for (int k = 0; k < 11; ++k)
    for (const char* p = ORC_POS3[k]; *p; ++p) c3[orc_letter(*p)] = k;
}

static int64_t orc_len(const int64_t* seq_start, int32_t pad, int32_t i) {
  return seq_start[i + 1] - seq_start[i] - pad;
}

/* Stage 0: key_off[8801], occ_seq/occ_pos ascending (seq, pos) within a key.
 * Returns the number of words. */
int64_t orc_build_index(const uint8_t* codes, const int64_t* seq_start, int32_t n_seqs, int32_t pad,
                        int64_t* key_off, int32_t* occ_seq, int32_t* occ_pos) {
  int c2[20], c3[20];
  orc_classes(c2, c3);
  int64_t* count = (int64_t*)calloc(ORC_NKEYS, sizeof(int64_t));
  for (int32_t s = 0; s < n_seqs; ++s) {
    const uint8_t* a = codes + seq_start[s];
    int64_t len = orc_len(seq_start, pad, s);
    for (int64_t p = 0; p + ORC_W <= len; ++p) {
      int key = ((a[p] * 2 + c2[a[p + 1]]) * 11 + c3[a[p + 2]]) * 20 + a[p + 3];
      count[key]++;
    }
  }
  key_off[0] = 0;
  for (int k = 0; k < ORC_NKEYS; ++k) key_off[k + 1] = key_off[k] + count[k];
  memset(count, 0, ORC_NKEYS * sizeof(int64_t));
  for (int32_t s = 0; s < n_seqs; ++s) {
    const uint8_t* a = codes + seq_start[s];
    int64_t len = orc_len(seq_start, pad, s);
    for (int64_t p = 0; p + ORC_W <= len; ++p) {
      int key = ((a[p] * 2 + c2[a[p + 1]]) * 11 + c3[a[p + 2]]) * 20 + a[p + 3];
      int64_t slot = key_off[key] + count[key]++;
      occ_seq[slot] = s;
      occ_pos[slot] = (int32_t)p;
    }
  }
  int64_t total = key_off[ORC_NKEYS];
  free(count);
  return total;
}

typedef struct {
  const uint8_t* codes;
  const int64_t* seq_start;
  int32_t n_seqs, pad;
  const int64_t* key_off;
  const int32_t* occ_seq;
  const int32_t* occ_pos;
} orc_bank_t;

/* Score of one pair: best rightward prefix over min(right, remaining) letters
 * plus best leftward prefix over min(nbr, available) letters. */
static int orc_pair_score(const orc_bank_t* A, int32_t s1, int32_t p1, const orc_bank_t* B, int32_t s2,
                          int32_t p2, const int8_t* mat, int nbr, int right) {
  const uint8_t* a = A->codes + A->seq_start[s1];
  const uint8_t* b = B->codes + B->seq_start[s2];
  int64_t la = orc_len(A->seq_start, A->pad, s1), lb = orc_len(B->seq_start, B->pad, s2);
  int64_t rmax = right;
  if (la - p1 < rmax) rmax = la - p1;
  if (lb - p2 < rmax) rmax = lb - p2;
  int s = 0, best_r = 0;
  for (int64_t t = 0; t < rmax; ++t) {
    s += mat[a[p1 + t] * 20 + b[p2 + t]];
    if (s > best_r) best_r = s;
  }
  int64_t lmax = nbr;
  if (p1 < lmax) lmax = p1;
  if (p2 < lmax) lmax = p2;
  s = 0;
  int best_l = 0;
  for (int64_t t = 1; t <= lmax; ++t) {
    s += mat[a[p1 - t] * 20 + b[p2 - t]];
    if (s > best_l) best_l = s;
  }
  return best_r + best_l;
}

typedef struct {
  const orc_bank_t *A, *B;
  const int8_t* mat;
  int32_t s1, nbr, right;
  const int32_t* keys;
  int32_t n_keys;
  int64_t next;          /* shared key counter */
  int64_t n_hits;        /* shared output cursor */
  int64_t n_ext;
  int32_t* out;
  int64_t cap;
  pthread_mutex_t lock;
} orc_job_t;

static void orc_flush(orc_job_t* J, const int32_t* buf, int64_t n) {
  pthread_mutex_lock(&J->lock);
  int64_t at = J->n_hits;
  J->n_hits += n;
  pthread_mutex_unlock(&J->lock);
  for (int64_t h = 0; h < n; ++h)
    if (at + h < J->cap) memcpy(J->out + 5 * (at + h), buf + 5 * h, 5 * sizeof(int32_t));
}

static void* orc_worker(void* arg) {
  orc_job_t* J = (orc_job_t*)arg;
  int64_t bufcap = 4096, nbuf = 0, ext = 0;
  int32_t* buf = (int32_t*)malloc(bufcap * 5 * sizeof(int32_t));
  for (;;) {
    int64_t q = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
    if (q >= J->n_keys) break;
    int32_t k = J->keys ? J->keys[q] : (int32_t)q;
    for (int64_t i = J->A->key_off[k]; i < J->A->key_off[k + 1]; ++i) {
      for (int64_t j = J->B->key_off[k]; j < J->B->key_off[k + 1]; ++j) {
        int sc = orc_pair_score(J->A, J->A->occ_seq[i], J->A->occ_pos[i], J->B, J->B->occ_seq[j],
                                J->B->occ_pos[j], J->mat, J->nbr, J->right);
        ++ext;
        if (sc >= J->s1) {
          if (nbuf == bufcap) {
            orc_flush(J, buf, nbuf);
            nbuf = 0;
          }
          int32_t* r = buf + 5 * nbuf++;
          r[0] = J->A->occ_seq[i];
          r[1] = J->A->occ_pos[i];
          r[2] = J->B->occ_seq[j];
          r[3] = J->B->occ_pos[j];
          r[4] = sc;
        }
      }
    }
  }
  orc_flush(J, buf, nbuf);
  free(buf);
  __atomic_fetch_add(&J->n_ext, ext, __ATOMIC_RELAXED);
  return NULL;
}

/* Stage 2 over the listed keys (all keys when keys == NULL).  Writes at most
 * cap hit rows (seq1, pos1, seq2, pos2, score) in unspecified order and returns
 * the total number of hits; *n_ext receives the number of pairs scored. */
int64_t orc_ungapped(const uint8_t* codes1, const int64_t* start1, int32_t n1, const int64_t* key_off1,
                     const int32_t* occ_seq1, const int32_t* occ_pos1, const uint8_t* codes2,
                     const int64_t* start2, int32_t n2, const int64_t* key_off2, const int32_t* occ_seq2,
                     const int32_t* occ_pos2, int32_t pad, const int8_t* mat, int32_t s1, int32_t nbr,
                     int32_t right, const int32_t* keys, int32_t n_keys, int32_t nthreads, int32_t* out,
                     int64_t cap, int64_t* n_ext) {
  orc_bank_t A = {codes1, start1, n1, pad, key_off1, occ_seq1, occ_pos1};
  orc_bank_t B = {codes2, start2, n2, pad, key_off2, occ_seq2, occ_pos2};
  orc_job_t J;
  memset(&J, 0, sizeof(J));
  J.A = &A;
  J.B = &B;
  J.mat = mat;
  J.s1 = s1;
  J.nbr = nbr;
  J.right = right;
  J.keys = keys;
  J.n_keys = keys ? n_keys : ORC_NKEYS;
  J.out = out;
  J.cap = cap;
  pthread_mutex_init(&J.lock, NULL);
  if (nthreads < 1) nthreads = 1;
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
  for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, orc_worker, &J);
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(th);
  pthread_mutex_destroy(&J.lock);
  if (n_ext) *n_ext = J.n_ext;
  return J.n_hits;
}

/* ------------------------------------------------------------------ gapped */

#define ORC_NEG (-(1 << 28))

/* Anchored banded affine-gap DP over x[0..lx) and y[0..ly) read with strides
 * dx, dy (+1 rightward, -1 leftward).  Cell (i, j) exists iff i <= lx, j <= ly
 * and |i - j| <= band.  Gap of length k costs open + k*ext.
 * Returns max(0, best H over existing cells). */
static int orc_gapped_side(const uint8_t* x, int lx, int dx, const uint8_t* y, int ly, int dy,
                           const int8_t* mat, int band, int open, int ext) {
  int W1 = ly + 1;
  int* H = (int*)malloc(sizeof(int) * (lx + 1) * W1);
  int* E = (int*)malloc(sizeof(int) * (lx + 1) * W1);
  int* F = (int*)malloc(sizeof(int) * (lx + 1) * W1);
  int best = 0;
  for (int i = 0; i <= lx; ++i) {
    for (int j = 0; j <= ly; ++j) {
      int c = i * W1 + j;
      H[c] = E[c] = F[c] = ORC_NEG;
      if ((i > j ? i - j : j - i) > band) continue;
      if (i == 0 && j == 0) {
        H[c] = 0;
        continue;
      }
      if (j >= 1 && (i > j - 1 ? i - (j - 1) : (j - 1) - i) <= band) {
        int e1 = E[c - 1] - ext, e2 = H[c - 1] - open - ext;
        E[c] = e1 > e2 ? e1 : e2;
      }
      if (i >= 1 && ((i - 1) > j ? (i - 1) - j : j - (i - 1)) <= band) {
        int f1 = F[c - W1] - ext, f2 = H[c - W1] - open - ext;
        F[c] = f1 > f2 ? f1 : f2;
      }
      int h = ORC_NEG;
      if (i >= 1 && j >= 1) h = H[c - W1 - 1] + mat[x[(i - 1) * dx] * 20 + y[(j - 1) * dy]];
      if (E[c] > h) h = E[c];
      if (F[c] > h) h = F[c];
      if (h < ORC_NEG) h = ORC_NEG;
      H[c] = h;
      if (h > best) best = h;
    }
  }
  free(H);
  free(E);
  free(F);
  return best;
}

typedef struct {
  const orc_bank_t *A, *B;
  const int32_t* hits;
  int64_t n;
  const int8_t* mat;
  int32_t window, band, open, ext;
  int32_t* gscore;
  int64_t next;
} orc_gjob_t;

static void* orc_gworker(void* arg) {
  orc_gjob_t* J = (orc_gjob_t*)arg;
  for (;;) {
    int64_t h = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
    if (h >= J->n) break;
    const int32_t* r = J->hits + 5 * h;
    int32_t s1 = r[0], p1 = r[1], s2 = r[2], p2 = r[3];
    const uint8_t* a = J->A->codes + J->A->seq_start[s1];
    const uint8_t* b = J->B->codes + J->B->seq_start[s2];
    int64_t la = orc_len(J->A->seq_start, J->A->pad, s1), lb = orc_len(J->B->seq_start, J->B->pad, s2);
    int rx = (int)(la - p1 < J->window ? la - p1 : J->window);
    int ry = (int)(lb - p2 < J->window ? lb - p2 : J->window);
    int lx = p1 < J->window ? p1 : J->window;
    int ly = p2 < J->window ? p2 : J->window;
    int right = orc_gapped_side(a + p1, rx, 1, b + p2, ry, 1, J->mat, J->band, J->open, J->ext);
    int left = orc_gapped_side(a + p1 - 1, lx, -1, b + p2 - 1, ly, -1, J->mat, J->band, J->open, J->ext);
    J->gscore[h] = right + left;
  }
  return NULL;
}

void orc_gapped(const uint8_t* codes1, const int64_t* start1, const uint8_t* codes2, const int64_t* start2,
                int32_t pad, const int32_t* hits, int64_t n, const int8_t* mat, int32_t window, int32_t band,
                int32_t open, int32_t ext, int32_t nthreads, int32_t* gscore) {
  orc_bank_t A = {codes1, start1, 0, pad, 0, 0, 0};
  orc_bank_t B = {codes2, start2, 0, pad, 0, 0, 0};
  orc_gjob_t J = {&A, &B, hits, n, mat, window, band, open, ext, gscore, 0};
  if (nthreads < 1) nthreads = 1;
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
  for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, orc_gworker, &J);
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(th);
}
