// Device image of a packed term program, shared by the host packer and the kernels.
//
// The paper stores each subterm as a row (dummy flag, 4 alpha/pi, P^psi bits, 4 beta/pi,
// P^phi bits) and lays the table out column-major for coalescing (Section 3.3, Appendix D).
// Here the same information is re-laid for one lane per assignment: the affine forms of all
// factors become a bit-vector L(x) of F bits (W 32-bit words), one column per parameter
// holds the forms that contain it (so a Gray-code step updates L with W XORs), and the
// factors are summarised by a few weighted popcount masks over L (value classes).  Every
// offset below counts 32-bit words from the start of the image; the int64 value table sits
// at a byte offset aligned to 8.
#pragma once

#include <stdint.h>

// statistics computed per term from popcounts of L (see the packer for their meaning)
enum { STAT_A = 0, STAT_B = 1, STAT_E = 2, STAT_R = 3, N_STATS = 4 };

struct ImgHeader {
    uint32_t pe;        // parameters enumerated by the kernel (p plus one per pair factor)
    uint32_t g;         // Gray-walk bits: packed positions 0 .. g-1
    uint32_t W;         // 32-bit words per form vector
    uint32_t has_zero;  // some factor can vanish: test the zero masks
    uint32_t has_mono;  // variable monomials present
    uint32_t n_slices_lo, n_slices_hi;  // 2^(pe - g)
    uint32_t off_col;   // pe * W words: forms containing packed position j
    uint32_t off_cvec;  // W words: constant bits of the forms
    uint32_t off_z0;    // W words: forms whose factor vanishes when the form is 0
    uint32_t off_z1;    // W words: ... when the form is 1
    uint32_t stat_off[N_STATS];  // entries of (W + 1) words: weight, mask[W]
    uint32_t stat_n[N_STATS];
    int32_t stat_base[N_STATS];
    uint32_t off_monohi;  // monomials over high positions only: c, mask_lo, mask_hi (slice bits)
    uint32_t n_monohi;
    uint32_t off_didx;    // g + 1 words: delta entries for walk position i are [didx[i], didx[i+1])
    uint32_t off_delta;   // entries of 4 words: c, walk mask, slice mask lo, slice mask hi
    uint32_t table_byte_off;  // int64 table: 4 coefficients per entry
    uint32_t table_n;         // entries
    int32_t d_off;            // table index of (d, r, e) = ((d + d_off) * 8 + r) * 2 + e
    uint32_t zero_entry;      // index of the all-zero entry
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
