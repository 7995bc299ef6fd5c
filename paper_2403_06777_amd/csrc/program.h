// Term programs: the IR text, its parser and printer, and the packer that turns a program
// into the device image evaluated by the kernels.
#pragma once

#include <string>
#include <vector>

#include "image.h"
#include "zw.h"

// A program denotes S = sqrt2^e * c * sum_x w^{phi(x)} prod_j F_j(x) (the parametric scalar
// of Eq. 2, one decomposition term per assignment x of the p Boolean parameters).
struct IrForm {
    int cst;        // constant bit
    uint64_t mask;  // bit i = parameter x_i enters the parity
};
struct IrNode {
    int form, a, b;  // 1 + w^{a + b l(x)}   (the node subterm; b = 4 for 1 + e^{i(alpha + pi l)})
};
struct IrPair {
    int f1, f2, a, b;  // 1 + w^{a + 4 l1} + w^{b + 4 l2} - w^{a + b + 4(l1 xor l2)}   (Eq. 3)
};
struct IrLin {
    int c, form;  // phi += c l(x)
};
struct IrMono {
    int c;
    std::vector<int> vars;  // phi += c prod x_v
};

struct IrProgram {
    int p = 0;
    int outer = 0;  // the last `outer` parameters are query parameters (kept as top slice bits)
    std::vector<IrForm> forms;
    std::vector<IrNode> nodes;
    std::vector<IrPair> pairs;
    std::vector<IrLin> lin;
    std::vector<IrMono> mono;
    Zw scalar = zw_one();
    int32_t e = 0;
};

// A product of affine forms with a Z/8 coefficient: phi += c * l_1(x) ... l_d(x) (d = 2 or 3).
// Variable monomials become such products when the exact elimination of the vanishing
// conditions substitutes an affine form for a parameter; they never appear in IR text.
struct IrFormMono {
    int c;
    std::vector<IrForm> forms;
};

bool ir_parse(const char *text, size_t len, IrProgram *out, std::string *err);
std::string ir_print(const IrProgram &prog);

struct PackedProgram {
    ImgHeader hdr;
    std::vector<uint8_t> blob;  // image words, padding, int64 value table
    std::vector<int32_t> perm;  // bit j of a slice-ordered index is parameter perm[j]
    int p = 0;                  // parameters of the program (terms = 2^p)
    int q = 0;                  // pair factors turned into walk parameters
    int walk_bits = 0;          // original parameters enumerated inside a slice
    int outer = 0;              // query parameters: the top `outer` bits of a slice index
    uint64_t n_slices = 1;
    Zw c0 = zw_one();           // constant, canonical
    int32_t e = 0;
    bool zero = false;          // a constant factor vanished
    int n_factors = 0, n_mono = 0, n_forms = 0;
    int W = 1;
    double ops_per_term = 0.0;  // algorithmic int32 lane-ops per term (see pack_program)
    double nonzero_fraction = 1.0;  // exact fraction of assignments where no factor vanishes
    // exact elimination of the vanishing conditions (pack_program): the program as given has
    // p_given parameters; `eliminated` of them were solved for, so the kernel sums over the
    // 2^p (p = p_given - eliminated) surviving assignments x = x0 XOR sum_j t_j cols[j], t the
    // slice-ordered index (cols and x0 are assignments of the given parameters)
    int p_given = 0;
    int eliminated = 0;
    uint64_t lay_x0 = 0;
    std::vector<uint64_t> lay_cols;
    int n_fmono = 0, n_mforms = 0;
};

// Returns 0 or a negative SIM_E* code with *err set.  max_walk_bits caps the Gray walk.
// eliminate: solve the vanishing conditions exactly (see eliminate_vanishing in the packer);
// false keeps them as factors tested at run time
int pack_program(const IrProgram &ir, int max_walk_bits, PackedProgram *out, std::string *err,
                 bool eliminate = true);

// exact value of one table entry: w^r * sqrt2^e * (1 + w)^d (d >= 0) or (1 + w^3)^(-d)
Zw table_value(int d, int r, int e);
