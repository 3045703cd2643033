// Stage 0, bank indexing (Sec. 3.3.1): subset-seed key of every word, then a
// stable sort by key into CSR form (key_off, occ, occ_seq).
//
// Pass 1's counting kernel also validates the bank against its layout and
// writes the scan codes (the letters scaled to table offsets) that the
// extension kernels read.
//
// The sort is a two-pass LSD radix sort on the 14-bit key: the low 7 bits
// (128 buckets), then the high 7 bits (69 buckets).  Each pass cuts its input
// into tiles of kIxTile elements, one wavefront each (four per workgroup): a
// counting kernel writes the tile's bucket histogram bucket-major, an
// exclusive scan over (bucket, tile) gives every tile its first slot in each
// bucket, and a scattering kernel ranks the tile's elements in order within
// their bucket (one ballot per digit bit over the 64 lanes of a round) into the
// tile's own bucket order in LDS, then writes the staged tile out bucket by
// bucket, consecutive lanes on consecutive slots.  Both passes are stable, so
// the order inside a key is the position order: ascending (sequence,
// position), independent of scheduling.  Pass 1 reads the codes (staged in
// LDS) and writes one 64-bit entry per word (position, key, and the sequence
// as an offset from the first sequence of the position's tile, which the
// layout check records per tile) and, beside it, the byte of its high digit
// that pass 2's counting kernel reads; pass 2 writes occ and occ_seq, and
// key_off follows from the two scanned histograms.
#include "plast_internal.h"

namespace plast {

namespace {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

constexpr int kIxTile = 2048;                       // elements per tile (32 rounds of 64)
constexpr int kIxWaves = 4;                         // tiles (one per wavefront) per workgroup
constexpr int kD0Bits = 7;                          // pass-1 digit: key & 127
constexpr int kD0 = 1 << kD0Bits;
constexpr int kD1 = (kNKeys + kD0 - 1) >> kD0Bits;  // pass-2 digit: key >> 7, 69 values
static_assert(kD1 <= 128, "pass-2 digits must fit 7 bits");

// Keeps the compiler from moving LDS accesses across a step of a wavefront's
// read-then-update of its own LDS table.  The lanes of a wavefront issue LDS
// instructions together and the LDS serves one wavefront's instructions in
// order, so no hardware barrier is needed.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Layout check, and the tile table: tile_seq[t] is the sequence holding
// position t * kIxTile (sequence 0 for the leading separators).  A sequence
// writes its tiles only when its own starts are consistent; the table is read
// only when no thread flagged the layout, and then every tile is written.
__global__ void k_layout_check(const int64_t* __restrict__ seq_start, int32_t n_seqs, int64_t n_padded,
                               int32_t* __restrict__ tile_seq, int64_t tiles, int32_t* __restrict__ err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n_seqs) return;
  int64_t s = seq_start[i];
  bool bad = s < kPadLen || s > n_padded;
  if (i == 0 && s != kPadLen) bad = true;
  if (i == n_seqs && s != n_padded) bad = true;
  if (i < n_seqs) {
    const int64_t nx = seq_start[i + 1];
    if (nx - s < kPadLen) bad = true;
    if (!bad) {
      const int64_t lo = i == 0 ? 0 : s;
      for (int64_t t = (lo + kIxTile - 1) / kIxTile; t < tiles && t * kIxTile < nx; ++t) tile_seq[t] = (int32_t)i;
    }
  }
  if (bad) atomicOr(err, 1);
}

// Loads starts s0 + 1 .. s0 + 64 * K of the sequences (INT64_MAX past the
// last) into a wavefront's LDS table, one coalesced load per 64.
template <int K>
__device__ __forceinline__ void load_starts(const int64_t* __restrict__ seq_start, int32_t n_seqs, int s0,
                                            int64_t* st, int lane) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t idx = (int64_t)s0 + 1 + k * 64 + lane;
    st[k * 64 + lane] = idx < n_seqs ? seq_start[idx] : INT64_MAX;
  }
}


// Lanes of the wavefront holding a valid element with the same 7-bit digit.
__device__ __forceinline__ uint64_t digit_peers(int d, bool valid) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 7; ++b) {
    const int bit = (d >> b) & 1;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

// A tile's bucket tables from the scanned histogram (bucket-major over
// tiles, n_total words in all): gst[d] is the tile's first slot in bucket d,
// lst[d] the first slot of bucket d in the tile's own bucket order, cur[d] a
// running copy of lst[d].  Returns the tile's word count.
template <int ND>
__device__ __forceinline__ int tile_tables(const int32_t* __restrict__ offs, int64_t tiles, int64_t tile,
                                           int64_t n_total, int32_t* gst, int32_t* lst, int32_t* cur, int lane) {
  int c[2], g[2], incl[2], tot[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int d = lane + 64 * h;
    g[h] = 0;
    c[h] = 0;
    if (d < ND) {
      const int64_t idx = (int64_t)d * tiles + tile;
      g[h] = offs[idx];
      c[h] = (int)((idx + 1 < (int64_t)ND * tiles ? (int64_t)offs[idx + 1] : n_total) - g[h]);
    }
    incl[h] = c[h];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl[h], o);
      if (lane >= o) incl[h] += t;
    }
    tot[h] = __shfl(incl[h], 63);
  }
  const int l0 = incl[0] - c[0], l1 = tot[0] + incl[1] - c[1];
  gst[lane] = g[0];
  gst[lane + 64] = g[1];
  lst[lane] = cur[lane] = l0;
  lst[lane + 64] = cur[lane + 64] = l1;
  return tot[0] + tot[1];
}

// Stable rank of the round's valid lanes within their digit: writes every
// valid lane's tile-local slot and advances the digit's running counter.
__device__ __forceinline__ int rank_in_tile(int d, bool valid, int32_t* cur, uint64_t below) {
  const uint64_t peers = digit_peers(d, valid);
  const int start = valid ? cur[d] : 0;
  wave_sync();
  const int l = start + __popcll(peers & below);
  if (valid && (peers & below) == 0) cur[d] = start + __popcll(peers);
  wave_sync();
  return l;
}

// The word arrays between the passes hold one 64-bit entry per word: the
// position (bits 0-31), the sequence as an offset from the first sequence of
// the position's pass-1 tile (bits 32-38) and the key (bits 39-52).
__device__ __forceinline__ uint64_t word_entry(int64_t q, int seq_off, int key) {
  return (uint64_t)(uint32_t)q | ((uint64_t)seq_off << 32) | ((uint64_t)key << 39);
}

// Pass 1, scattering.  The tile's codes are staged in LDS; every word, in
// position order, is ranked within its low digit into the tile's own bucket
// order in LDS (key | position offset << 14 | sequence offset << 25), and the
// staged words are then written out bucket by bucket, consecutive lanes to
// consecutive slots.  Runs only on a valid layout (the tile table is complete,
// a tile meets at most 103 sequence starts and the words fit the word array).
constexpr int kTileStarts = 2;  // 128 starts
static_assert(kIxTile == 2048, "word staging packs a position offset in 11 bits");

// A tile's codes [beg, beg + kIxTile + 64) into LDS as dwords (separators past
// n_padded), with dword loads when the codes are 4-byte aligned.
__device__ __forceinline__ void stage_codes(const uint8_t* __restrict__ codes, int64_t beg, int64_t n_padded,
                                            uint32_t* cl32, int lane) {
  const int nb = (int)max(min(n_padded - beg, (int64_t)(kIxTile + 64)), (int64_t)0);  // code bytes in range
  const bool aligned = (reinterpret_cast<uintptr_t>(codes) & 3) == 0;
#pragma unroll
  for (int r = 0; r < ((kIxTile + 64) / 4 + 63) / 64; ++r) {
    const int j = r * 64 + lane;
    if (j < (kIxTile + 64) / 4) {
      const int o = 4 * j;
      uint32_t v;
      if (aligned && o + 4 <= nb) {
        v = *(const uint32_t*)(codes + beg + o);
      } else {
        v = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) v |= (uint32_t)(o + k < nb ? codes[beg + o + k] : (uint8_t)kPadCode) << (8 * k);
      }
      cl32[j] = v;
    }
  }
}

// Seed key of the word whose four codes are the bytes of w, or -1 unless all
// four are residues (< 20).  ((w + 108 per byte) | w) has a byte's top bit set
// iff that byte is >= 20; a carry out of a byte comes only from a byte >= 148,
// which has its own top bit set.
__device__ __forceinline__ int word_key4(uint32_t w, const SeedClasses& sc) {
  if (((w + 0x6C6C6C6Cu) | w) & 0x80808080u) return -1;
  return seed_key_dev(sc, (int)(w & 0xffu), (int)((w >> 8) & 0xffu), (int)((w >> 16) & 0xffu), (int)(w >> 24));
}

// Seed key of the word starting at byte off of the staged codes (-1 unless all
// four codes are residues): two aligned dword reads and a funnel shift.
__device__ __forceinline__ int word_key_at(const uint32_t* cl32, int off, const SeedClasses& sc) {
  return word_key4(__builtin_amdgcn_alignbyte(cl32[(off >> 2) + 1], cl32[off >> 2], (uint32_t)(off & 3)), sc);
}

// Pass 1, counting, fused with the validation of the bank and the writing of
// the scan codes: one wavefront per tile of kIxTile positions (tiles past the
// bank write the scan codes' tail slack only).  The tile's codes (and the 64
// after it) are staged in LDS once.  Validation: position p is a residue iff
// some sequence s has seq_start[s] <= p < seq_start[s + 1] - kPadLen; residues
// must be < 20 and every other position below n_padded the separator.  The
// residue positions of the tile come as a bitmap: the state at the tile's first
// position, toggled at every sequence start and every residue end inside the
// tile (a sequence with no residue toggles twice at one position), resolved by
// a prefix xor within each lane's 32 positions and a prefix parity across the
// lanes.  The scan codes are the validated codes times kScale.  The histogram
// counts the low digit of the key of every word starting in the tile, from the
// raw codes, as the scattering pass does (four word starts per lane and round):
// on a valid bank a word of four codes < 20 lies inside one sequence.  After a
// layout error nothing is validated or written but the histogram.
__global__ __launch_bounds__(64 * kIxWaves) void k_ix_check_count1(
    const uint8_t* __restrict__ codes, const int64_t* __restrict__ seq_start, int32_t n_seqs, int64_t n_padded,
    const int32_t* __restrict__ tile_seq, int64_t tiles, uint8_t* __restrict__ scan, int64_t scan_len, SeedClasses sc,
    int32_t* __restrict__ hist, int32_t* __restrict__ err) {
  __shared__ int32_t cnt_all[kIxWaves][kD0];
  __shared__ uint32_t rb_all[kIxWaves][kIxTile / 32];
  __shared__ uint32_t cl_all[kIxWaves][(kIxTile + 64) / 4];
  const int lane = lane_id(), wv = threadIdx.x >> 6;
  const int64_t tile = (int64_t)blockIdx.x * kIxWaves + wv;
  const int64_t beg = tile * kIxTile;
  if (tile >= tiles && beg >= scan_len) return;
  int32_t* cnt = cnt_all[wv];
  uint32_t* rb = rb_all[wv];
  uint32_t* cl32 = cl_all[wv];
  stage_codes(codes, beg, n_padded, cl32, lane);
  cnt[lane] = 0;
  cnt[lane + 64] = 0;
  rb[lane] = 0;
  const bool layout_ok = !(*err & 1);
  wave_sync();
  if (layout_ok) {
    // s0: the last sequence with seq_start <= beg (-1 before the first one)
    int s0 = n_seqs - 1;
    if (beg < n_padded && n_seqs > 0) {
      s0 = min(max(tile_seq[min(tile, tiles - 1)], 0), n_seqs - 1);
      if (seq_start[s0] > beg) s0 = -1;
    }
    const bool init = s0 >= 0 && beg < (s0 + 1 < n_seqs ? seq_start[s0 + 1] : n_padded) - kPadLen;
    // Toggles from the starts s0 + 1 .. s0 + 128 (n_padded standing for
    // seq_start[n_seqs]): a start inside the tile, and the residue end kPadLen
    // before it.  A valid layout puts at most 104 of them within kIxTile + kPadLen
    // of beg, since consecutive starts are at least kPadLen apart.
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int64_t idx = (int64_t)s0 + 1 + k * 64 + lane;
      if (idx <= n_seqs) {
        const int64_t v = idx < n_seqs ? seq_start[idx] : n_padded;
        const int64_t e = v - kPadLen;
        if (idx < n_seqs && v > beg && v < beg + kIxTile) atomicXor(&rb[(v - beg) >> 5], 1u << ((v - beg) & 31));
        if (e > beg && e < beg + kIxTile) atomicXor(&rb[(e - beg) >> 5], 1u << ((e - beg) & 31));
      }
    }
    wave_sync();
    {
      const uint32_t tog = rb[lane];
      uint32_t x = tog;
      x ^= x << 1;
      x ^= x << 2;
      x ^= x << 4;
      x ^= x << 8;
      x ^= x << 16;
      const uint64_t odd = __ballot(__popc(tog) & 1);
      const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
      const bool flip = ((__popcll(odd & below) & 1) != 0) != init;
      rb[lane] = flip ? ~x : x;
    }
    wave_sync();
    bool bad = false;
    const int64_t vend = min(beg + kIxTile, scan_len);
    // 256 positions per round, four consecutive ones per lane (scan is
    // 256-byte aligned and scan_len a multiple of 256: one dword per lane)
    for (int64_t base = beg; base < vend; base += 256) {
      const int off = (int)(base - beg) + 4 * lane;
      const uint32_t raw = cl32[off >> 2];
      const uint32_t res = (rb[off >> 5] >> (off & 31)) & 15u;
      uint32_t out = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        uint32_t c = kPadCode;
        if (beg + off + k < n_padded) {
          const bool residue = (res >> k) & 1u;
          c = (raw >> (8 * k)) & 0xffu;
          bad |= residue ? (c >= 20) : (c != kPadCode);
          if (!(residue && c < 20)) c = kPadCode;
        }
        out |= (c * kScale) << (8 * k);
      }
      *(uint32_t*)(scan + beg + off) = out;
    }
    if (bad) atomicOr(err, 2);
  }
  if (tile >= tiles) return;
  const int nw = (int)(min(beg + kIxTile, n_padded - (kSeed - 1)) - beg);  // word starts [beg, beg + nw)
#pragma unroll 2
  for (int r = 0; r < kIxTile / 256; ++r) {
    const int o = r * 256 + 4 * lane;
    if (o < nw) {
      const uint32_t lo = cl32[o >> 2], hi = cl32[(o >> 2) + 1];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int key = word_key4(__builtin_amdgcn_alignbyte(hi, lo, k), sc);
        if (o + k < nw && key >= 0) atomicAdd(&cnt[key & (kD0 - 1)], 1);
      }
    }
  }
  wave_sync();
  hist[(int64_t)lane * tiles + tile] = cnt[lane];
  hist[(int64_t)(lane + 64) * tiles + tile] = cnt[lane + 64];
}

__global__ __launch_bounds__(64 * kIxWaves) void k_ix_scatter1(
    const uint8_t* __restrict__ codes, const int64_t* __restrict__ seq_start, int32_t n_seqs, int64_t n_padded,
    int64_t tiles, SeedClasses sc, const int32_t* __restrict__ tile_seq, const int32_t* __restrict__ err,
    const int32_t* __restrict__ offs, int64_t cap, uint64_t* __restrict__ words, uint8_t* __restrict__ digits) {
  __shared__ int32_t gst_all[kIxWaves][kD0], lst_all[kIxWaves][kD0], cur_all[kIxWaves][kD0];
  __shared__ int64_t st_all[kIxWaves][64 * kTileStarts];
  __shared__ uint32_t stage_all[kIxWaves][kIxTile];
  __shared__ uint32_t cl_all[kIxWaves][(kIxTile + 64) / 4];
  __shared__ uint32_t sbits_all[kIxWaves][kIxTile / 32], spre_all[kIxWaves][kIxTile / 32];
  const int lane = lane_id(), wv = threadIdx.x >> 6;
  const int64_t tile = (int64_t)blockIdx.x * kIxWaves + wv;
  if (tile >= tiles || n_seqs == 0 || (*err & 1)) return;
  int32_t *gst = gst_all[wv], *lst = lst_all[wv], *cur = cur_all[wv];
  int64_t* st = st_all[wv];
  uint32_t* stage = stage_all[wv];
  uint32_t* cl32 = cl_all[wv];
  uint32_t *sbits = sbits_all[wv], *spre = spre_all[wv];
  const int64_t beg = tile * kIxTile;
  const int64_t end = min(beg + kIxTile, n_padded - (kSeed - 1));  // word starts [beg, end)
  stage_codes(codes, beg, n_padded, cl32, lane);
  const int s0 = min(max(tile_seq[tile], 0), n_seqs - 1);
  load_starts<kTileStarts>(seq_start, n_seqs, s0, st, lane);
  sbits[lane] = 0;
  const int nt = tile_tables<kD0>(offs, tiles, tile, (int64_t)err[1], gst, lst, cur, lane);
  wave_sync();
  // The sequence of a position, s0 + the number of sequence starts in the tile
  // at or before it: a bitmap of the starts (one 32-bit word per lane; at most
  // 103 starts fall in a tile, all after its first position) and the count of
  // starts before each word.
#pragma unroll
  for (int k = 0; k < kTileStarts; ++k) {
    const int64_t o = st[k * 64 + lane] - beg;
    if (o > 0 && o < kIxTile) atomicOr(&sbits[o >> 5], 1u << (o & 31));
  }
  wave_sync();
  {
    const uint32_t b = sbits[lane];
    int incl = __popc(b);
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o);
      if (lane >= o) incl += t;
    }
    spre[lane] = (uint32_t)(incl - __popc(b));
  }
  wave_sync();
  auto seq_at = [&](int off) {  // off = position - beg, in [0, kIxTile)
    const int w = off >> 5;
    return s0 + (int)spre[w] + __popc(sbits[w] & (~0u >> (31 - (off & 31))));
  };
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  auto entry = [&](int key, int off, int s) {
    return (uint32_t)key | ((uint32_t)(off + lane) << 14) | ((uint32_t)min(s - s0, 127) << 25);
  };
  if (nt <= kIxTile / 2) {
    // Sparse tile (translated fragments: most positions are separators): the
    // words are first compacted in position order into the upper half of the
    // stage, then ranked from there into the lower half, ceil(nt / 64) rounds
    // instead of one per 64 positions; the halves do not overlap.
    // Four consecutive word starts per lane and round (two aligned dword reads);
    // a word's place is the valid words of the lanes below plus those of its
    // own lane before it, and its sequence the bitmap count at its position
    // (the four positions share one 32-bit word of the bitmap).
    uint32_t* comp = stage + kIxTile / 2;
    int nw = 0;
    const int nwp = (int)(end - beg);  // word starts in the tile (none if <= 0)
    for (int o0 = 0; o0 < nwp; o0 += 256) {
      const int o = o0 + 4 * lane;
      const uint32_t lo = cl32[o >> 2], hi = cl32[(o >> 2) + 1];
      int key[4];
      uint64_t bal[4];
      int before = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        key[k] = o + k < nwp ? word_key4(__builtin_amdgcn_alignbyte(hi, lo, (uint32_t)k), sc) : -1;
        bal[k] = __ballot(key[k] >= 0);
        before += __popcll(bal[k] & below);
      }
      const uint32_t sb = sbits[o >> 5];
      const int sp = s0 + (int)spre[o >> 5];
      int at = nw + before;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (key[k] >= 0) {
          const int s = sp + __popc(sb & (~0u >> (31 - ((o + k) & 31))));
          if (at < kIxTile / 2)
            comp[at] = (uint32_t)key[k] | ((uint32_t)(o + k) << 14) | ((uint32_t)min(s - s0, 127) << 25);
          ++at;
        }
      }
      nw += __popcll(bal[0]) + __popcll(bal[1]) + __popcll(bal[2]) + __popcll(bal[3]);
    }
    wave_sync();
    nw = min(nw, kIxTile / 2);
    for (int c = 0; c < nw; c += 64) {
      const bool valid = c + lane < nw;
      const uint32_t e = valid ? comp[c + lane] : 0u;
      const int l = rank_in_tile((int)(e & (kD0 - 1)), valid, cur, below);
      if (valid && (unsigned)l < (unsigned)(kIxTile / 2)) stage[l] = e;
    }
  } else {
    for (int off = 0; beg + off < end; off += 64) {
      const int64_t q = beg + off + lane;
      const int key = q < end ? word_key_at(cl32, off + lane, sc) : -1;
      const int l = rank_in_tile(key & (kD0 - 1), key >= 0, cur, below);
      if (key >= 0 && (unsigned)l < (unsigned)kIxTile) stage[l] = entry(key, off, seq_at(off + lane));
    }
  }
  wave_sync();
  for (int l = lane; l < min(nt, kIxTile); l += 64) {
    const uint32_t e = stage[l];
    const int key = (int)(e & 0x3fffu);
    const int d = key & (kD0 - 1);
    const int64_t slot = (int64_t)gst[d] + (l - lst[d]);
    if (slot >= 0 && slot < cap) {
      words[slot] = word_entry(beg + ((e >> 14) & 2047u), (int)(e >> 25), key);
      digits[slot] = (uint8_t)min(key >> kD0Bits, kD1 - 1);
    }
  }
}

// Pass 2, counting: histogram of the high digit over the tile's words, read
// from the byte per word that pass 1 writes beside each entry (four per lane
// and round; the array is 256-byte aligned and padded, so a dword that
// straddles the end stays inside it).
__global__ __launch_bounds__(64 * kIxWaves) void k_ix_count2(const uint8_t* __restrict__ digits,
                                                            const int32_t* __restrict__ err, int64_t cap,
                                                            int64_t tiles, int32_t* __restrict__ hist) {
  __shared__ int32_t cnt_all[kIxWaves][kD0];
  const int lane = lane_id();
  const int64_t tile = (int64_t)blockIdx.x * kIxWaves + (threadIdx.x >> 6);
  if (tile >= tiles || (*err & 1)) return;
  int32_t* cnt = cnt_all[threadIdx.x >> 6];
  cnt[lane] = 0;
  cnt[lane + 64] = 0;
  wave_sync();
  const int64_t n = min((int64_t)err[1], cap);
  const int64_t beg = tile * kIxTile;
  const int64_t end = min(beg + kIxTile, n);
  for (int64_t i = beg + 4 * lane; i < end; i += 256) {
    const uint32_t d4 = *(const uint32_t*)(digits + i);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (i + k < end) atomicAdd(&cnt[min((int)((d4 >> (8 * k)) & 0xffu), kD1 - 1)], 1);
  }
  wave_sync();
  if (lane < kD1) hist[(int64_t)lane * tiles + tile] = cnt[lane];
  if (lane + 64 < kD1) hist[(int64_t)(lane + 64) * tiles + tile] = cnt[lane + 64];
}

// Pass 2, scattering: the tile's words ranked within their high digit into
// the tile's bucket order in LDS, eight rounds of loads in flight ahead of
// the ranking, then written out bucket by bucket as occ and occ_seq, eight
// slots per lane at a time.
constexpr int kBatch = 8;

__global__ __launch_bounds__(64 * kIxWaves) void k_ix_scatter2(
    const uint64_t* __restrict__ words, const int32_t* __restrict__ tile_seq, int64_t tiles1,
    const int32_t* __restrict__ err, int64_t cap, int64_t tiles, const int32_t* __restrict__ offs, int32_t* __restrict__ occ,
    int32_t* __restrict__ occ_seq) {
  __shared__ int32_t gst_all[kIxWaves][kD0], lst_all[kIxWaves][kD0], cur_all[kIxWaves][kD0];
  __shared__ uint64_t stage_all[kIxWaves][kIxTile];
  const int lane = lane_id(), wv = threadIdx.x >> 6;
  const int64_t tile = (int64_t)blockIdx.x * kIxWaves + wv;
  if (tile >= tiles || (*err & 1)) return;
  int32_t *gst = gst_all[wv], *lst = lst_all[wv], *cur = cur_all[wv];
  uint64_t* stage = stage_all[wv];
  const int64_t n = min((int64_t)err[1], cap);
  const int64_t beg = tile * kIxTile;
  const int64_t end = min(beg + kIxTile, n);
  const int nt = tile_tables<kD1>(offs, tiles, tile, n, gst, lst, cur, lane);
  wave_sync();
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint64_t e_cur[kBatch], e_nxt[kBatch];
#pragma unroll
  for (int k = 0; k < kBatch; ++k) {
    const int64_t i = beg + k * 64 + lane;
    e_cur[k] = i < end ? words[i] : 0;
  }
  for (int64_t b0 = beg; b0 < end; b0 += 64 * kBatch) {
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      const int64_t i = b0 + (kBatch + k) * 64 + lane;
      e_nxt[k] = i < end ? words[i] : 0;
    }
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      const bool valid = b0 + k * 64 + lane < end;
      const int l = rank_in_tile(min((int)(e_cur[k] >> (39 + kD0Bits)), kD1 - 1), valid, cur, below);
      if (valid && (unsigned)l < (unsigned)kIxTile) stage[l] = e_cur[k];
    }
#pragma unroll
    for (int k = 0; k < kBatch; ++k) e_cur[k] = e_nxt[k];
  }
  wave_sync();
  // eight slots per lane at a time, so that their tile-table loads are in
  // flight together
  const int nl = min(nt, kIxTile);
  for (int l0 = 0; l0 < nl; l0 += 64 * kBatch) {
    uint64_t e[kBatch];
    int32_t ts[kBatch];
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      const int l = l0 + k * 64 + lane;
      e[k] = l < nl ? stage[l] : 0;
    }
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      const uint32_t t1 = (uint32_t)e[k] >> 11;
      ts[k] = (int64_t)t1 < tiles1 ? tile_seq[t1] : -1;
    }
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      const int l = l0 + k * 64 + lane;
      if (l >= nl) continue;
      const int key = (int)(e[k] >> 39);
      const int d = min(key >> kD0Bits, kD1 - 1);
      const int64_t slot = (int64_t)gst[d] + (l - lst[d]);
      if (slot < 0 || slot >= n) continue;
      occ[slot] = (int32_t)(uint32_t)e[k];
      occ_seq[slot] = ts[k] >= 0 ? ts[k] + (int)((e[k] >> 32) & 127u) : -1;
    }
  }
}

__global__ void k_clear2(int32_t* __restrict__ p) {
  if (threadIdx.x < 2) p[threadIdx.x] = 0;
}

// key_off from the two scanned histograms, with no pass over the sorted words.
// After pass 1 the word array is ordered by the low digit: the words whose low
// digit is below lo are its first offs1[lo * tiles1] entries.  Pass 2 cuts that
// array into tiles of kIxTile entries, and its scanned histogram holds, for
// high digit d and tile t, the words of high digit below d plus those of high
// digit d in the tiles before t.  So the words with key below k = d * 128 + lo
// number offs2[d * tiles2 + t] for the tile t holding entry offs1[lo * tiles1],
// plus the words of high digit d in that tile before the entry, which one
// workgroup per low digit counts (fewer than kIxTile entries).  A key with no
// word gets the first slot of the next key that has one, n_words past the
// last.  After a layout error the index holds no word.
__global__ __launch_bounds__(256) void k_ix_key_off(const uint64_t* __restrict__ words,
                                                    const int32_t* __restrict__ offs1, int64_t tiles1,
                                                    const int32_t* __restrict__ offs2, int64_t tiles2,
                                                    const int32_t* __restrict__ err, int64_t cap,
                                                    int64_t* __restrict__ key_off) {
  __shared__ int32_t cnt[kD1];
  const int lo = blockIdx.x;
  const bool none = (err[0] & 1) != 0;
  const int64_t n = none ? 0 : min((int64_t)err[1], cap);
  for (int d = threadIdx.x; d < kD1; d += blockDim.x) cnt[d] = 0;
  __syncthreads();
  const int64_t start = none ? 0 : min(max((int64_t)offs1[(int64_t)lo * tiles1], (int64_t)0), n);
  const int64_t t = start / kIxTile;
  for (int64_t i = t * kIxTile + threadIdx.x; i < start; i += blockDim.x)
    atomicAdd(&cnt[min((int)(words[i] >> (39 + kD0Bits)), kD1 - 1)], 1);
  __syncthreads();
  for (int d = threadIdx.x; d < kD1; d += blockDim.x) {
    const int k = d * kD0 + lo;
    if (k >= kNKeys) continue;
    int64_t v = 0;
    if (!none) {
      const int64_t idx = (int64_t)d * tiles2 + t;
      v = min((idx < (int64_t)kD1 * tiles2 ? (int64_t)offs2[idx] : n) + cnt[d], n);
    }
    key_off[k] = v;
  }
  if (lo == 0 && threadIdx.x == 0) key_off[kNKeys] = n;
}

// ---------------------------------------------------------------- scan
constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanBlock = kScanThreads * kScanPer;

__device__ __forceinline__ int block_excl_scan(int v, int* total) {
  __shared__ int wsum[kScanThreads / 64];
  int lane = lane_id(), wid = threadIdx.x / 64;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) {
    before += (w < wid) ? wsum[w] : 0;
    all += wsum[w];
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_local(int32_t* __restrict__ data, int64_t n,
                                                             int32_t* __restrict__ tops) {
  int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  int v[kScanPer];
  int sum = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    v[i] = (base + i < n) ? data[base + i] : 0;
    sum += v[i];
  }
  int total;
  int run = block_excl_scan(sum, &total);
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    if (base + i < n) data[base + i] = run;
    run += v[i];
  }
  if (threadIdx.x == 0) tops[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tops(int32_t* __restrict__ tops, int64_t nb,
                                                            int32_t* __restrict__ grand) {
  int carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kScanBlock) {
    int64_t base = b0 + (int64_t)threadIdx.x * kScanPer;
    int v[kScanPer];
    int sum = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
      v[i] = (base + i < nb) ? tops[base + i] : 0;
      sum += v[i];
    }
    int total;
    int run = carry + block_excl_scan(sum, &total);
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
      if (base + i < nb) tops[base + i] = run;
      run += v[i];
    }
    carry += total;
  }
  if (threadIdx.x == 0 && grand) *grand = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int32_t* __restrict__ data, int64_t n,
                                                           const int32_t* __restrict__ tops) {
  int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  int add = tops[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanPer; ++i)
    if (base + i < n) data[base + i] += add;
}

}  // namespace

size_t scan_tmp_bytes(int64_t n) { return align_up(sizeof(int32_t) * (size_t)((n + kScanBlock - 1) / kScanBlock + 1), 256); }

void exclusive_scan_i32(int32_t* d_data, int64_t n, int32_t* d_total, void* d_tmp, hipStream_t s) {
  int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb == 0) nb = 1;
  int32_t* tops = (int32_t*)d_tmp;
  hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kScanThreads), 0, s, d_data, n, tops);
  hipLaunchKernelGGL(k_scan_tops, dim3(1), dim3(kScanThreads), 0, s, tops, nb, d_total);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, d_data, n, (const int32_t*)tops);
}

IndexLayout index_layout(int64_t n_padded) {
  IndexLayout L;
  size_t off = 0;
  L.key_off = off;
  off = align_up(off + sizeof(int64_t) * (kNKeys + 1), 256);
  L.occ = off;
  off = align_up(off + sizeof(int32_t) * (size_t)n_padded, 256);
  L.occ_seq = off;
  off = align_up(off + sizeof(int32_t) * (size_t)n_padded, 256);
  L.scan = off;
  off = align_up(off + (size_t)n_padded + kScanSlack, 256);
  L.total = off;
  return L;
}

// Workspace: [error words (256 B)] [tile table] [pass-1 histogram] [pass-2 histogram]
// [scan scratch] [word entries between the passes (64-bit)] [their high digits (8-bit)].
// The word arrays hold n_padded - kPadLen entries, a bound on the residues of any valid
// layout that grows with n_padded alone, so a workspace sized for the largest
// bank serves every smaller one whatever its number of sequences.
struct IxWs {
  int64_t tiles1, tiles2, cap;
  size_t tile_seq, hist1, hist2, tmp, words, digits, total;
};

IxWs ix_ws(int64_t n_padded) {
  IxWs w;
  w.cap = n_padded > kPadLen ? n_padded - kPadLen : 0;
  w.tiles1 = (n_padded + kIxTile - 1) / kIxTile;
  if (w.tiles1 < 1) w.tiles1 = 1;
  w.tiles2 = (w.cap + kIxTile - 1) / kIxTile;
  if (w.tiles2 < 1) w.tiles2 = 1;
  size_t off = 256;
  w.tile_seq = off;
  off = align_up(off + sizeof(int32_t) * (size_t)w.tiles1, 256);
  w.hist1 = off;
  off = align_up(off + sizeof(int32_t) * (size_t)(kD0 * w.tiles1), 256);
  w.hist2 = off;
  off = align_up(off + sizeof(int32_t) * (size_t)(kD1 * w.tiles2), 256);
  w.tmp = off;
  const int64_t scan_n = kD0 * w.tiles1 > kD1 * w.tiles2 ? kD0 * w.tiles1 : kD1 * w.tiles2;
  off = align_up(off + scan_tmp_bytes(scan_n), 256);
  w.words = off;
  off = align_up(off + sizeof(uint64_t) * (size_t)w.cap, 256);
  w.digits = off;
  off = align_up(off + (size_t)w.cap, 256);
  w.total = off;
  return w;
}

size_t index_ws_bytes(int64_t n_padded) { return ix_ws(n_padded).total; }

int index_enqueue(const uint8_t* d_codes, const int64_t* d_seq_start, int32_t n_seqs, int64_t n_padded,
                  void* d_index, void* d_ws, int32_t* d_err, plast_index_t* out, hipStream_t stream) {
  IndexLayout L = index_layout(n_padded);
  const IxWs W = ix_ws(n_padded);
  uint8_t* base = (uint8_t*)d_index;
  int64_t* key_off = (int64_t*)(base + L.key_off);
  int32_t* occ = (int32_t*)(base + L.occ);
  int32_t* occ_seq = (int32_t*)(base + L.occ_seq);
  uint8_t* scan = base + L.scan;
  int64_t scan_len = (int64_t)(L.total - L.scan);

  uint8_t* ws = (uint8_t*)d_ws;
  int32_t* total = d_err + 1;
  int32_t* tile_seq = (int32_t*)(ws + W.tile_seq);
  int32_t* hist1 = (int32_t*)(ws + W.hist1);
  int32_t* hist2 = (int32_t*)(ws + W.hist2);
  void* tmp = ws + W.tmp;
  uint64_t* words = (uint64_t*)(ws + W.words);
  uint8_t* digits = ws + W.digits;

  SeedClasses sc = seed_classes();
  timing_mark(kStageIndex, false, stream);
  // a fill kernel rather than a memset node, so that the sequence can be captured in a graph
  hipLaunchKernelGGL(k_clear2, dim3(1), dim3(64), 0, stream, d_err);
  hipLaunchKernelGGL(k_layout_check, dim3((unsigned)((n_seqs + 1 + 255) / 256)), dim3(256), 0, stream, d_seq_start,
                     n_seqs, n_padded, tile_seq, W.tiles1, d_err);
  // After a layout error the passes that read the tile table or the word
  // arrays return at once and key_off says the index holds no word.
  const unsigned g1 = (unsigned)((W.tiles1 + kIxWaves - 1) / kIxWaves);
  const unsigned g2 = (unsigned)((W.tiles2 + kIxWaves - 1) / kIxWaves);
  const int64_t tiles_scan = (scan_len + kIxTile - 1) / kIxTile;  // tiles covering the scan codes and their slack
  const int64_t tiles_c = tiles_scan > W.tiles1 ? tiles_scan : W.tiles1;
  hipLaunchKernelGGL(k_ix_check_count1, dim3((unsigned)((tiles_c + kIxWaves - 1) / kIxWaves)), dim3(64 * kIxWaves), 0,
                     stream, d_codes, d_seq_start, n_seqs, n_padded, (const int32_t*)tile_seq, W.tiles1, scan,
                     scan_len, sc, hist1, d_err);
  exclusive_scan_i32(hist1, kD0 * W.tiles1, total, tmp, stream);
  hipLaunchKernelGGL(k_ix_scatter1, dim3(g1), dim3(64 * kIxWaves), 0, stream, d_codes, d_seq_start, n_seqs,
                     n_padded, W.tiles1, sc, (const int32_t*)tile_seq, (const int32_t*)d_err, (const int32_t*)hist1,
                     W.cap, words, digits);
  hipLaunchKernelGGL(k_ix_count2, dim3(g2), dim3(64 * kIxWaves), 0, stream, (const uint8_t*)digits,
                     (const int32_t*)d_err, W.cap, W.tiles2, hist2);
  exclusive_scan_i32(hist2, kD1 * W.tiles2, nullptr, tmp, stream);
  hipLaunchKernelGGL(k_ix_scatter2, dim3(g2), dim3(64 * kIxWaves), 0, stream, (const uint64_t*)words,
                     (const int32_t*)tile_seq, W.tiles1, (const int32_t*)d_err, W.cap, W.tiles2,
                     (const int32_t*)hist2, occ, occ_seq);
  hipLaunchKernelGGL(k_ix_key_off, dim3(kD0), dim3(256), 0, stream, (const uint64_t*)words, (const int32_t*)hist1,
                     W.tiles1, (const int32_t*)hist2, W.tiles2, (const int32_t*)d_err, W.cap, key_off);
  timing_mark(kStageIndex, true, stream);
  PLAST_HIP(hipGetLastError());

  out->codes = d_codes;
  out->seq_start = d_seq_start;
  out->n_seqs = n_seqs;
  out->n_padded = n_padded;
  out->key_off = key_off;
  out->occ = occ;
  out->occ_seq = occ_seq;
  out->scan_codes = scan;
  out->n_words = -1;
  return PLAST_OK;
}

int build_index_impl(const uint8_t* d_codes, const int64_t* d_seq_start, int32_t n_seqs, int64_t n_padded,
                     void* d_index, void* d_ws, plast_index_t* out, hipStream_t stream) {
  int32_t* err = (int32_t*)d_ws;  // [0] error bits, [1] word total
  plast_index_t view;
  int rc = index_enqueue(d_codes, d_seq_start, n_seqs, n_padded, d_index, d_ws, err, &view, stream);
  if (rc != PLAST_OK) return rc;
  int32_t h_err[2] = {0, 0};
  PLAST_HIP(hipMemcpyAsync(h_err, err, sizeof(h_err), hipMemcpyDeviceToHost, stream));
  PLAST_HIP(hipStreamSynchronize(stream));
  if (h_err[0] & 1) return set_error(PLAST_E_LAYOUT, "seq_start does not describe the padded layout");
  if (h_err[0] & 2) return set_error(PLAST_E_ALPHABET, "a residue code is > 19 or a separator code is not 20");
  view.n_words = h_err[1];
  *out = view;
  return PLAST_OK;
}

}  // namespace plast
