// Sparse stage of the decomposition: parallel-vector rounding of sparse unfoldings.
#pragma once

#include "common.hpp"

namespace tts {

// Bit layout of the packed coordinate key: the field of mode j (0-based) sits at
// bit off[j] with width bits[j]; mode 0 is least significant, so the last mode is
// most significant and every suffix (i_{k+1},...,i_d) is a contiguous high part.
struct ModeInfo {
  int32_t d;
  uint32_t bits[TT_MAX_D];
  uint32_t off[TT_MAX_D];
  uint32_t n[TT_MAX_D];
};

// Small device-side status block, read back once or twice per level.
struct DevStatus {
  uint32_t err;       // bit 0: index out of range, bit 1: non-finite, bit 2: duplicate
  uint32_t table_over;  // a grouping table too small for its level (speculative pass)
  uint32_t ncols;     // columns of the current level
  uint32_t beta;      // groups of the current level
  uint32_t nnz_n;     // entries of N_k
  uint32_t dropped;   // explicit zeros among the input entries
  unsigned long long longmask;  // bit k - 1: a level-k column has more than kMaxLocal entries
  double norm2;       // ||A||_F^2
};

constexpr uint32_t kErrIndex = 1u, kErrNonfinite = 2u, kErrDuplicate = 4u;
constexpr int kMaxLocal = 32;  // longest column canonicalised from registers
// levels of at most this many columns (rows not yet ordered) take one wave per column
constexpr uint32_t kCanonWaveMax = 4096;
// probes per column in a speculative pass's grouping table (at most a quarter full
// while the speculation holds)
constexpr uint32_t kSpecMaxProbe = 32;

// a1: validate, drop zeros (key := ~0), pack keys; values copied as raw bits.
void launch_ingest(const int32_t* idx, const double* val, uint32_t nnz, const ModeInfo& mi,
                   uint64_t* keys, uint64_t* vbits, DevStatus* st, hipStream_t s);

// Column starts of a level: flag[e] = 1 where (ekey[e] >> sh) changes.  Level 1
// also checks duplicates and accumulates ||A||^2 (fixed-order partial sums).
// long_bit >= 0: set bit long_bit of st->longmask if a column has more than kMaxLocal
// entries (one bit per level, so that nothing needs clearing between levels).
void launch_col_flags(const uint64_t* ekey, uint32_t nE, int sh, bool level1, int long_bit,
                      const double* ev, uint32_t* flag, double* norm_part, DevStatus* st, hipStream_t s);
uint32_t norm_partials_count(uint32_t nE);
void launch_norm_final(const double* part, uint32_t np, DevStatus* st, hipStream_t s);
void launch_col_starts(const uint32_t* flag, const uint32_t* pos, uint32_t nE, uint32_t* col_start,
                       const uint32_t* d_ncols, hipStream_t s);
// The same three steps in two launches without flag arrays (tiles of 4096 entries, at
// most kStartsMaxTiles of them), with level 1's duplicate check and per-tile sums of
// squares into norm_part[starts_tiles(nE)] (level1), or the long-column bit
// (long_bit >= 0); part holds starts_tiles(nE) words.
constexpr uint32_t kStartsMaxTiles = 4096;
uint32_t starts_tiles(uint32_t nE);
void launch_starts(const uint64_t* ekey, uint32_t nE, int sh, bool level1, int long_bit, const double* ev,
                   uint32_t* part, double* norm_part, uint32_t* col_start, uint32_t* d_ncols, DevStatus* st,
                   hipStream_t s);
// The same three steps (flags, scan, starts) for a level k >= 2 of 1 .. kColsSmallMax
// entries in one workgroup; the flags and places themselves are not kept.
constexpr uint32_t kColsSmallMax = 16384;
void launch_columns_small(const uint64_t* ekey, uint32_t nE, int sh, int long_bit, uint32_t* col_start,
                          uint32_t* d_ncols, DevStatus* st, hipStream_t s);
// Column counts of every level from the sorted kept keys, and the duplicate flag; see
// k_level_counts.  Level k's count is the sum of counts[k * kLevelCountCopies + c],
// c < kLevelCountCopies (k = 1 .. d-1, all (d + 1) * kLevelCountCopies words zeroed
// beforehand).
constexpr uint32_t kLevelCountCopies = 32;
void launch_level_counts(const uint64_t* keys, uint32_t n, const ModeInfo& mi, uint32_t* counts, DevStatus* st,
                         hipStream_t s);

// Long-column path: composite sort keys (column << rbits | rho) and a permutation.
void launch_make_composite(const uint32_t* flag, const uint32_t* pos, const uint32_t* erho, uint32_t nE,
                           int rbits, uint64_t* ckey, uint64_t* cval, hipStream_t s);
void launch_permute_entries(const uint64_t* perm, uint32_t nE, const uint64_t* ekey_in, const uint32_t* erho_in,
                            const double* ev_in, uint64_t* ekey_out, uint32_t* erho_out, double* ev_out,
                            hipStream_t s);

struct CanonArgs {
  const uint64_t* ekey;
  const uint32_t* erho;  // null at level 1 (rho = low field of ekey)
  const double* ev;
  const uint32_t* col_start;
  uint32_t ncols;
  int sh;               // bits of mode k-1 (0-based): column = ekey >> sh
  uint64_t rho_mask;    // level 1: mask of the mode-0 field
  int kidx;             // first suffix mode (0-based) = k
  bool sort_rows;       // entries of a column still need ordering by rho
  int snap;             // fraction bits dropped from every canonical value (0: exact test)
  uint32_t* crho;       // out, per entry: rho in ascending order
  double* cval;         // out, per entry: canonical value v / s
  uint64_t* colhash;
  double* cols;         // prefactor s
  uint64_t* colsuf;     // colex-packed suffix (lowest field = mode k)
  uint64_t* rmkey;      // row-major-ordered suffix key (numbering order)
  // the grouping's hash table (tsize slots), cleared here for the next step: table to
  // 0 (empty), slotmin to ~0 (no minimum yet)
  uint64_t* table;
  uint64_t* slotmin;
  uint32_t tsize;
  uint32_t* slot_gid;  // tsize group ids, cleared to 0 here too (may be null)
};
// a4: canonicalise every column by its entry of smallest row, key and hash it.
// wide: one workgroup per column (for levels of few, long columns already in row
// order); otherwise one lane per column.
void launch_canon(const CanonArgs& a, const ModeInfo& mi, DevStatus* st, bool wide, hipStream_t s);

// a5: group identical canonical columns (open-addressing table of tmask + 1 slots with
// full-key verification), leader = smallest row-major suffix key of each group.  A
// column probes at most max_probe slots; one that finds neither its group nor an
// empty slot sets *over (when given) and is left without a group.  A table with more
// slots than columns and max_probe = its size never overflows.
void launch_group(const uint64_t* colhash, const uint32_t* crho, const double* cval, const uint32_t* col_start,
                  const uint64_t* rmkey, uint32_t ncols, uint64_t* table, uint64_t* slotmin, uint32_t tmask,
                  uint32_t max_probe, uint32_t* over, uint32_t* slot, uint32_t* isrep, hipStream_t s);
// the leaders' (row-major key, slot) pairs at their group positions below cap
void launch_rep_list(const uint32_t* isrep, const uint32_t* reppos, const uint32_t* slot, const uint64_t* slotmin,
                     uint32_t ncols, uint32_t cap, uint64_t* lkey, uint64_t* lslot, hipStream_t s);
// group id of each slot (= rank of its leader) and the length of each group's column,
// for entries j < n of nlen, n = *d_beta when given (then zero for beta <= j < n),
// else beta
void launch_group_ids(const uint64_t* lslot_sorted, uint32_t beta, const uint32_t* d_beta, uint32_t n,
                      const uint64_t* table, const uint32_t* col_start, uint32_t* slot_gid, uint32_t* nlen,
                      hipStream_t s);

// The leaders of at most cap (<= kSmallSortMax) groups in one workgroup: ordered by
// row-major key (stable rank sort), numbered (slot_gid of each slot = its leader's
// rank), and the lengths of their columns scanned into npos with the total in *d_nnz;
// lss = the slots in group order.  The list is either given (lkey, lslot: beta =
// *d_beta entries, as launch_rep_list writes them), or built here: from a table of
// at most kLeaderTableMax slots (tscan: an occupied slot is a group, its minimum the
// leader's key; the list in slot order, *d_beta written), or for at most
// kLeaderListMax columns (isrep non-null) from the columns' flags, slots and slot
// minima, with *d_beta and each representative's place reppos written too.  More
// than cap groups: nothing written beyond *d_beta and reppos.
constexpr uint32_t kLeaderListMax = 16384;
constexpr uint32_t kLeaderTableMax = 8192;
struct LeaderArgs {
  int tscan;       // build the list from the table (tsize slots)
  uint32_t tsize;
  const uint32_t* isrep;  // non-null: build the list from the columns
  uint32_t* reppos;
  const uint32_t* slot;
  const uint64_t* slotmin;
  uint32_t ncols;
  const uint64_t* lkey;  // else: the given list
  const uint64_t* lslot;
  uint32_t* d_beta;
  uint32_t cap;
  int nbits;  // key bits compared
  const uint64_t* table;
  const uint32_t* col_start;
  uint64_t* lss;
  uint32_t* slot_gid;
  uint32_t* npos;
  uint32_t* d_nnz;
};
void launch_leaders(const LeaderArgs& a, hipStream_t s);

struct EmitArgs {
  uint32_t ncols;
  const uint32_t* slot;
  const uint32_t* slot_gid;
  const uint64_t* colsuf;
  const double* cols;
  int kidx;            // first suffix mode (0-based)
  bool last;           // k == d-1: write the last core
  // keep_intermediates (may be null)
  int64_t* out_col;
  int32_t* out_g;
  double* out_s;
  // next level (k < d-1)
  uint64_t* next_ekey;
  uint32_t* next_rho;
  double* next_v;
  // last level: dense G^(d) [beta][n_d], zero-filled beforehand
  double* last_core;
  // N_k: the groups' slots in group order (lss), their columns' places (npos)
  const uint64_t* lss;
  uint32_t bmax;  // groups the launch covers
  const uint32_t* d_beta;
  const uint32_t* d_nnz;
  const uint64_t* table;
  const uint32_t* col_start;
  const uint32_t* npos;
  const uint32_t* crho;
  const double* cval;
  int64_t* colptr;
  int32_t* nrow;
  double* nval;
};
// a6 + a7 in one launch: N_k in CSC (one canonical column per group, in group order;
// beta = *d_beta, nnz(N_k) = *d_nnz; nothing written if beta > bmax), and the
// transfer matrix -> next level's entries (or the last core).
void launch_emit(const EmitArgs& a, const ModeInfo& mi, hipStream_t s);


}  // namespace tts
