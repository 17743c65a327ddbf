// Row-pass instances (see NTTK_FWD_ROWS in kernels_impl.hpp): compiled once per direction
// (NTTK_ROWS_DIR: 0 forward, 1 inverse, 2 key product), arithmetic policy (NTTK_ROWS_FAST)
// and range of row lengths [NTTK_ROWS_LO, NTTK_ROWS_HI] (log2 of the row length).
#include "kernels_impl.hpp"

#if NTTK_ROWS_DIR == 0
#define NTTK_INST(LM) NTTK_FWD_ROWS(, NTTK_ROWS_FAST, LM)
#elif NTTK_ROWS_DIR == 1
#define NTTK_INST(LM) NTTK_INV_ROWS(, NTTK_ROWS_FAST, LM)
#else
#define NTTK_INST(LM) NTTK_MUL_ROWS(, NTTK_ROWS_FAST, LM)
#endif

namespace nttk {
#if NTTK_ROWS_LO <= 1 && NTTK_ROWS_HI >= 1
NTTK_INST(1)
#endif
#if NTTK_ROWS_LO <= 2 && NTTK_ROWS_HI >= 2
NTTK_INST(2)
#endif
#if NTTK_ROWS_LO <= 3 && NTTK_ROWS_HI >= 3
NTTK_INST(3)
#endif
#if NTTK_ROWS_LO <= 4 && NTTK_ROWS_HI >= 4
NTTK_INST(4)
#endif
#if NTTK_ROWS_LO <= 5 && NTTK_ROWS_HI >= 5
NTTK_INST(5)
#endif
#if NTTK_ROWS_LO <= 6 && NTTK_ROWS_HI >= 6
NTTK_INST(6)
#endif
#if NTTK_ROWS_LO <= 7 && NTTK_ROWS_HI >= 7
NTTK_INST(7)
#endif
#if NTTK_ROWS_LO <= 8 && NTTK_ROWS_HI >= 8
NTTK_INST(8)
#endif
#if NTTK_ROWS_LO <= 9 && NTTK_ROWS_HI >= 9
NTTK_INST(9)
#endif
#if NTTK_ROWS_LO <= 10 && NTTK_ROWS_HI >= 10
NTTK_INST(10)
#endif
#if NTTK_ROWS_LO <= 11 && NTTK_ROWS_HI >= 11
NTTK_INST(11)
#endif
#if NTTK_ROWS_LO <= 12 && NTTK_ROWS_HI >= 12
NTTK_INST(12)
#endif
#if NTTK_ROWS_LO <= 13 && NTTK_ROWS_HI >= 13
NTTK_INST(13)
#endif
}  // namespace nttk
