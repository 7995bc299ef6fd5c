// Host-side compiler: Clifford+T circuit and query -> term program (IR).
#pragma once

#include <string>

#include "../../include/zxpar.h"
#include "program.h"

struct CompileOptions {
    int p_cap = 48;
    bool eliminate_constraints = true;
    bool hub_params = true;  // a parameter may go to any spider (see sim_compile_opts)
};

struct CompileStats {
    int t_count = 0;        // T-like spiders left after Clifford simplification
    int n_constraints = 0;  // parameters removed by parity constraints
    int n_params = 0;
};

// Returns SIM_OK or a negative SIM_E* code with *err set.
int compile_circuit(const char *text, size_t len, const sim_query &q, const CompileOptions &opts,
                    IrProgram *out, CompileStats *stats, std::string *err);
