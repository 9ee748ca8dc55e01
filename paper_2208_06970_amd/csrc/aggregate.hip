// placeholder, replaced below
#include "common.h"
extern "C" size_t lsrvt_aggregate_workspace(lsrvt_dims, uint32_t, uint32_t, int32_t, int32_t, int32_t, uint32_t) { return 256; }
extern "C" int32_t lsrvt_aggregate(const uint32_t *, lsrvt_dims, const uint32_t *, const uint32_t *, uint32_t, const uint8_t *,
                        uint32_t, int32_t, const float *, int32_t, const float *, int32_t, uint32_t,
                        const lsrvt_cell_stats *, const lsrvt_group_stats *, const lsrvt_group_stats *, void *, size_t, void *) { return LSRVT_EINVAL; }
