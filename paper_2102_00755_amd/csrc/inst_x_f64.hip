#define FWI_T double
#include "inst_x.inc"
