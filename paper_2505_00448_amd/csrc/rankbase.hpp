// Per-column sorted orders of a samples x variables matrix (the Spearman
// sort): layout shared by the Spearman scan, the subset queries and the rank
// tests.
#pragma once

#include "napy_internal.hpp"

namespace napy {

struct SpearBase {
    uint16_t* ord;     // [F][ld]
    uint16_t* ord2;    // [F][ld]: 2 x ord, the byte offset of each sample's entry in a uint16 array
                       //     indexed by sample (columns sorted in LDS only, S <= SORT_LDS_MAX_S)
    uint16_t* pos;     // [F][ld]
    uint32_t* runs;    // [F][ld]
    uint64_t* tbits;   // [F][ld/64]: bit k set if sorted position k lies in a tie run
    uint32_t* rlist;   // [F][ld/2]: tie run r (length > 1) of the column as s | e << 16
    int32_t* nruns;    // [F] number of tie runs
    int32_t* ncol;     // [F]
    int32_t* hasties;  // [F]
    int32_t* tcount;   // [F] number of positions in tie runs
    int32_t* perm;     // [F] processing order of the columns (see k_perm)
    int32_t* tcls;     // [F] tie class: 0 no ties, 1 few short runs, 2 otherwise (see k_tcls)
    int32_t* nsing;    // [F] untied observed positions of a densely tied column whose tie runs and
                       //     untied positions number at most RUN_GROUPS_MAX, else -1 (see k_tcls)
    uint16_t* sing;    // [F][RUN_GROUPS_MAX] those untied positions, ascending
    int64_t ld;
};

// Row stride of the per-column arrays: room for every sample plus one dummy
// sample index S whose position is always "missing", padded to whole groups
// of four 64-position chunks, so sorted-order reads past a column's observed
// count need no bounds test.
inline int64_t spear_ld(int64_t S) { return round_up(S + 1, 256); }
// sorted orders may be read up to this many entries past the last row
constexpr int64_t ORD_TAIL = 512;
// Columns of up to SORT_LDS_MAX_S samples are sorted in LDS (their sorted
// positions keep a tie flag in bit 15); longer ones, up to SPEAR_MAX_S (16-bit
// sample indices and positions, 0xFFFF meaning "missing"), over global
// memory, with positions only.
constexpr int64_t SORT_LDS_MAX_S = 24576;
constexpr int64_t SPEAR_MAX_S = 65535;
// 32-bit words of the keys buffer the sort uses: one plane of F x ld keys, or
// four (keys and sample indices, twice) for long columns
inline int64_t sort_keys_words(int64_t S, int64_t F) { return F * spear_ld(S) * (S > SORT_LDS_MAX_S ? 4 : 1); }
// value groups (tie runs plus untied positions) of a column whose ranks the
// pair scan takes from a per-partner table in LDS
constexpr int RUN_GROUPS_MAX = 23;

inline void base_carve(Carver& c, int64_t S, int64_t F, SpearBase& b)
{
    b.ld = spear_ld(S);
    b.ord = c.take<uint16_t>((size_t)F * b.ld + ORD_TAIL);
    b.ord2 = c.take<uint16_t>((size_t)F * b.ld + ORD_TAIL);
    b.pos = c.take<uint16_t>((size_t)F * b.ld);
    b.runs = c.take<uint32_t>((size_t)F * b.ld);
    b.tbits = c.take<uint64_t>((size_t)F * (b.ld / 64));
    b.rlist = c.take<uint32_t>((size_t)F * (b.ld / 2));
    b.nruns = c.take<int32_t>(F);
    b.ncol = c.take<int32_t>(F);
    b.hasties = c.take<int32_t>(F);
    b.tcount = c.take<int32_t>(F);
    b.perm = c.take<int32_t>(F);
    b.tcls = c.take<int32_t>(F);
    b.nsing = c.take<int32_t>(F);
    b.sing = c.take<uint16_t>((size_t)F * RUN_GROUPS_MAX);
}

// Sorts the columns of X into a base in `base` (spearman_base_bytes(S, F)
// bytes, carved by base_carve then a keys buffer).  Defined in spearman.hip.
int spearman_base_prepare_run(const float* X, int64_t S, int64_t F, int64_t ldx, void* base,
                              const napy_opts* opts, hipStream_t st);
size_t spearman_base_bytes(int64_t S, int64_t F);

}  // namespace napy
