#include "internal.h"
extern "C" qtt_status qtt_assemble_stiffness(const qtt_problem *, double, qtt_tt *, qtt_tt *, void *, size_t, void *) { return QTT_E_UNSUPPORTED; }
extern "C" qtt_status qtt_assemble_workspace(const qtt_problem *, size_t *, int64_t *, int64_t *) { return QTT_E_UNSUPPORTED; }
