#include "internal.h"
extern "C" qtt_status qtt_solve(const qtt_tt *, const qtt_tt *, const qtt_tt *, const qtt_solve_opts *, qtt_tt *, qtt_solve_report *, void *, size_t, void *) { return QTT_E_UNSUPPORTED; }
extern "C" qtt_status qtt_solve_workspace(const qtt_tt *, const qtt_tt *, const qtt_solve_opts *, size_t *) { return QTT_E_UNSUPPORTED; }
