#define FWI_T double
#include "inst_axis.inc"
