// Device image of a packed term program, shared by the host packer and the kernels.
//
// The paper stores each subterm as a row (dummy flag, 4 alpha/pi, P^psi bits, 4 beta/pi,
// P^phi bits) and lays the table out column-major for coalescing (Section 3.3, Appendix D).
// Here the same information is re-laid for one lane per slice of assignments: the affine
// forms of all factors become a bit-vector L(x) of F bits (W 32-bit words), one column per
// parameter holds the forms that contain it (so a Gray-code step updates L with W XORs), and
// the factors are summarised by weighted popcount masks over L (value classes).  Every offset
// below counts 32-bit words from the start of the image; the int64 value table sits at a
// byte offset aligned to 8.
#pragma once

#include <stdint.h>

// statistics computed per term from popcounts of L (see the packer for their meaning)
enum { STAT_A = 0, STAT_B = 1, STAT_E = 2, STAT_R = 3, N_STATS = 4 };

#ifdef __HIPCC__
#define IMG_HD __host__ __device__
#else
#define IMG_HD
#endif

// fixed statistic slots: A+1, A-1, B+1, B-1, E+1, E+2, E-1, E-2, R*1, R*2, R*4
constexpr int kSlots = 11;
IMG_HD constexpr int slot_stat(int i) { return i < 2 ? STAT_A : i < 4 ? STAT_B : i < 8 ? STAT_E : STAT_R; }
IMG_HD constexpr int slot_weight(int i) {
    return i == 0 ? 1 : i == 1 ? -1 : i == 2 ? 1 : i == 3 ? -1 : i == 4 ? 1 : i == 5 ? 2 : i == 6 ? -1
         : i == 7 ? -2 : i == 8 ? 1 : i == 9 ? 2 : 4;
}

// Menu of compile-time slot sets: a kernel variant computes exactly the slots of its set
// (branch-free); the packer picks the smallest set that covers the program's active slots
// and leaves the other slots of that set with zero masks.
constexpr uint32_t kSlotSetAll = 0x7FFu;    // every slot
constexpr uint32_t kSlotSetNodes = 0x7C5u;  // A+1, B+1, E-1, E-2, R*: factors 1 + w^{k l}
constexpr uint32_t kSlotSetPhase = 0x700u;  // R* only: phase terms without factors
constexpr uint32_t kSlotSetPhaseLow = 0x300u;  // R*1, R*2: phase terms beside the node table
// Added to the low phase set: the node factors are looked up in a table indexed by their bits
// (at most kMaxTableNodes node factors, bits 0 .. n-1 of word 0, then the bit of the one
// combined weight-4 phase term), whose entry holds the term's vanishing flag, A - B (offset), E
// and the part of R from the nodes and from the linear terms on those bits; the R*1 and R*2
// slots count the other linear terms (all their weight-4 parts are in that combined term).
constexpr uint32_t kSlotsNodeTable = 0x40000000u;
constexpr int kMaxTableNodes = 10;
IMG_HD constexpr uint32_t slot_set_of(uint32_t menu_index) {
    return menu_index == 1 ? kSlotSetNodes
         : menu_index == 2 ? kSlotSetPhase
         : menu_index == 3 ? (kSlotSetPhaseLow | kSlotsNodeTable)
                           : kSlotSetAll;
}
// Added to a slot set: the node-factor slots (A, B, E) and the R*4 slot have bits in word 0
// only, so they read one word; the R*1 and R*2 slots read all W.  The node bits come first,
// and the R*4 weights sit on them and on the one combined weight-4 phase term that follows
// them, so at most 31 node factors qualify.
constexpr uint32_t kSlotsNodeWord0 = 0x80000000u;
IMG_HD constexpr int slot_words(uint32_t set, int slot, int W) {
    return (set & kSlotsNodeWord0) && (slot_stat(slot) != STAT_R || slot_weight(slot) == 4) ? 1 : W;
}

// Walk positions 0 .. KB-1 (the inner bits) are stepped in unrolled blocks of 2^KB terms: the
// flip positions inside a block are compile-time constants, and the phase of every term of a
// block relative to its first term is one 4-bit field (mod 8) of a per-lane vector of
// 2^KB / 8 words built once per block.  Everything done once per block (the flip between
// blocks, the vanishing test) is spread over 2^KB terms: 32 for form vectors of up to 4
// words, 16 for wider ones (whose unrolled block keeps 2^KB columns of W words in registers).
// Programs with fewer walk bits use the plain step loop.
constexpr int kMaxInnerBits = 6;
// the most dynamic LDS (value table and the other tables) a program's kernels may take
constexpr unsigned kMaxDynLdsBytes = 64 * 1024;
// slots of the table of surviving steps (4 words each: key, 64-bit step mask, 0), for blocks of
// 2^KB steps: enough that a collision-free multiplier is found quickly for 2^KB keys
#ifdef __HIPCC__
__host__ __device__
#endif
constexpr uint32_t ztab_slots_for(int KB) { return KB >= 6 ? 512u : 256u; }
#ifdef __HIPCC__
__host__ __device__
#endif
constexpr int inner_bits_for(uint32_t W) { return W <= 2 ? 6 : W <= 4 ? 5 : 4; }

// how the terms of a lane are summed
enum {
    ACC_I64 = 0,   // every partial sum fits int64 (static bound): four int64 registers
    ACC_I128 = 1,  // four int128 registers, term shifted into them
    ACC_CLASS = 2  // per-block LDS counters of sum 2^h per value class, times the table at flush
};

struct ImgHeader {
    uint32_t pe;        // parameters enumerated by the kernel (p plus one per pair factor)
    uint32_t g;         // Gray-walk bits: packed positions 0 .. g-1
    uint32_t W;         // 32-bit words per form vector
    uint32_t has_zero;  // some factor can vanish: test the zero masks
    uint32_t has_mono;  // variable monomials present
    uint32_t acc;       // ACC_* mode
    uint32_t slot_menu; // index into the slot-set menu (0 all, 1 node factors, 2 phase only,
                        // 3 phase with the node table)
    uint32_t ntab_n;    // node table entries (2^node factors), 0 without the table
    uint32_t off_ntab;  // ntab_n words: bit 0 vanishes, bits 1-7 A - B + d_off, bits 8-15 E,
                        // bits 16-18 the node part of R (mod 8)
    uint32_t ntab_lds;  // byte offset of the node table in dynamic LDS
    uint32_t ztab_bits; // z > 0: the z vanishing bits all lie in word 0, and at off_ztab come a
    uint32_t ztab_mult; //   table of ztab_slots_for(KB) (key, mask lo, mask hi, 0) entries and
    uint32_t off_ztab;  //   the 2^KB values of P(gray(k)), W words each, P(y) = XOR of the inner
    uint32_t ztab_lds;  //   columns picked by y.  A block whose first term has a = L & zmask reads
    uint32_t ztab_shift;//   the entry at slot (a * ztab_mult) >> ztab_shift: if its key is a, bit k
                        //   of its mask says whether step k survives, else none does (the
                        //   multiplier maps the at most 2^KB values P(gray(k)) & zmask to
                        //   distinct slots).  Both tables are copied to dynamic LDS at byte
                        //   offset ztab_lds.
    uint32_t node_word0;  // the node-factor slot masks are zero beyond word 0
    uint32_t block_sum32; // int64 mode, node factors + KB <= 30: a lane's block of terms sums below 2^31
    uint32_t n_slices_lo, n_slices_hi;  // 2^(pe - g)
    uint32_t off_col;   // pe * W words: forms containing packed position j
    uint32_t off_cvec;  // W words: L at the all-zero assignment
    uint32_t off_zmask; // W words: bits of factors that can vanish; such a bit of L is 1 exactly
                        // where its factor vanishes (the form, complemented if that is at l = 0)
    uint32_t off_never; // W words: a value of L & zmask that no block's surviving terms have
    uint32_t inner_rank;  // rank r of the inner columns on the vanishing bits (walks of at least
    uint32_t off_ibasis;  //   KB positions): r entries of 3 + W words (pivot word, pivot bit,
                          //   inner columns making it up, reduced basis vector) and KB - r
                          //   all-zero entries (they change nothing), then at
    uint32_t off_ikern;   //   off_ikern the KB - r null-space combinations of the inner columns
    uint32_t off_slots; // kSlots entries of (W + 1) words: weight (0 = unused), mask[W]
    int32_t stat_base[N_STATS];
    uint32_t off_monohi;  // monomials over high positions only: c, mask_lo, mask_hi (slice bits)
    uint32_t n_monohi;
    // Gray-step changes of the variable monomials.  At a flip of walk position i the walk bits
    // below i are fixed (bit i-1 set, lower bits clear), so each monomial containing i either
    // always contributes when i flips, never does, or depends on walk bits above i:
    uint32_t off_ui;      // g words: sum of coefficients always firing with no slice part
    uint32_t off_aidx;    // g + 1 words: slice-dependent always-firing entries of position i are
    uint32_t off_al;      //   [aidx[i], aidx[i+1]) at off_al, 3 words each: c, slice mask lo, hi
    uint32_t off_didx;    // g + 1 words: walk-state-dependent entries of position i are
    uint32_t off_delta;   //   [didx[i], didx[i+1]) at off_delta, 4 words each (16-byte
                          //   aligned): c, walk mask (positions above i), slice mask lo, hi
    // Inner-block phase vectors, NF = 2^KB / 8 words each.  Field k (bits 4(k mod 8) .. +3 of
    // word k / 8) of a vector holds, mod 8, the phase of step k of a block minus that of step 0;
    // the walk state of step k inside the block is gray(k) on the inner positions, with the top
    // inner bit inverted in odd blocks, so every vector comes as an (even, odd) pair.  Only
    // monomials with an inner variable contribute; one is active when its other variables are
    // all 1:
    uint32_t off_inner;   // 2 NF words: sum over monomials whose other variables are all inner
    uint32_t off_c2;      // n_c2 entries, 2 NF + 2 words: even[NF], odd[NF], slice mask lo, hi
    uint32_t n_c2;        //   (other variables: slice bits only)
    uint32_t off_c3idx;   // g + 1 words: entries of outer walk position i (some other variable
    uint32_t off_c3;      //   is an outer walk bit) are [c3idx[i], c3idx[i+1]) at off_c3, each
    uint32_t n_c3;        //   4 NF words (aligned): even[NF], odd[NF], its other outer walk bits,
                          //   slice mask lo, hi, zeros; at a flip of i with the other bits set it
                          //   toggles on or off
    uint32_t off_pos;     // g records of 4 words (16-byte aligned), one per walk position i:
                          //   ui[i], didx[i] | didx[i+1] << 16, c3idx[i] | c3idx[i+1] << 16, 0
                          //   (what a flip of i reads, in one load)
    // A walk may start at any block of a slice (the work of a wave is a contiguous range of
    // blocks); its start state then needs:
    uint32_t off_c3all;   // n_c3all entries, 2 NF + 3 words: the inner-and-outer monomials once
    uint32_t n_c3all;     //   each (even[NF], odd[NF], outer walk mask, slice mask lo, hi)
    uint32_t off_monowalk;  // n_monowalk entries, 4 words: every monomial with a walk part
    uint32_t n_monowalk;    //   (c, walk mask, slice mask lo, hi)
    // Form monomials (products of two or three affine forms, left by the exact elimination of
    // the vanishing conditions).  Their n_mforms <= 32 distinct forms are the bits of a per-lane
    // vector O: at the first term of a block O = S ^ G ^ (odd block ? gcol_top : 0), S the forms'
    // constants and slice parts (per lane and slice), G their outer walk parts (uniform, xor of
    // gcol[i] over the set walk bits i; gcol[i] is word 3 of position i's record), and at step k
    // of the block a form is its bit of O xor bit k of its lambda.
    uint32_t n_fmono;
    uint32_t off_fmono;   // 8 words each: c | deg << 8 | j1 << 16 | j2 << 24, j3, lambda lo/hi x 3
    uint32_t n_mforms;
    uint32_t off_fmgrp;   // 15 words: entries [grp[k], grp[k + 1]) have 2 (k < 7) or 3 forms and
                          // coefficient k % 7 + 1 (the entries are sorted so)
    uint32_t off_fmh;     // term_split 2: 16 words of group bounds (two-form groups d2[0..7],
    uint32_t fmh_stride;  //   three-form groups d3[0..7], each group padded with null entries
    uint32_t fmh_off3;    //   to 8 or 4 entries), then two half tables (steps 0..31, 32..63)
                          //   fmh_stride words apart: two-form entries of 4 words (j1, j2,
                          //   lambda1, lambda2: that half's pattern word), then at fmh_off3
                          //   three-form entries of 8 words (j1, j2, j3, lambda1..3, 0, 0);
    uint32_t fmh_lds;     //   all copied to dynamic LDS at byte offset fmh_lds
    uint32_t off_mforms;  // 4 words each: slice mask lo, hi, constant, 0
    uint32_t off_scol;    // pe - g words: the forms containing slice bit j (S = fm_s0 ^ the
    uint32_t fm_s0;       //   columns of the set slice bits)
    uint32_t off_gcol;    // g words: the forms containing walk position i
    uint32_t gcol_top;    // gcol[KB - 1]: the top inner bit, set at the first term of odd blocks
    uint32_t block_flush128;  // int64 mode: each block's sums move to int128 after the block
    uint32_t term_split;      // 2: two waves share each unit, each taking half of a 64-term block
                              // (small programs with form monomials only); 1 otherwise
    uint32_t table_byte_off;  // int64 table: 4 coefficients per entry
    uint32_t table_n;         // entries (value classes + one zero entry)
    int32_t d_off;            // class of (d, r, e) = ((d + d_off) * 8 + r) * 2 + e
    uint32_t zero_entry;      // index of the all-zero entry (= number of classes)
    uint32_t q_limbs;         // ACC_CLASS: counters per class (2^h split as 2^(32 q) * 2^(h mod 32))
    uint32_t image_bytes;     // total bytes of the image
};

// one 64-byte partial sum: four int128 coefficients as (lo, hi) pairs
struct Partial {
    uint64_t w[8];
};

// a batch work item: slices [s_begin, s_end) of program prog, partial written to out_slot
struct WorkItem {
    uint32_t prog;
    uint32_t out_slot;
    uint64_t s_begin;
    uint64_t s_end;
};
