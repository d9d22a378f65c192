// placeholder translation unit (replaced by the batched executor)
#include <hip/hip_runtime.h>
