#include "compiler.h"

int compile_circuit(const char *, size_t, const sim_query &, const CompileOptions &, IrProgram *, CompileStats *,
                    std::string *err) {
    *err = "compiler not built yet";
    return SIM_EINVAL;
}
