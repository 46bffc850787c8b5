#define FWI_T float
#include "inst_x.inc"
