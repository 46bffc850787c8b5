#define FWI_T float
#include "inst_axis.inc"
