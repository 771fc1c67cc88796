// Time coupling (timecoupling.cpp).
#pragma once

#include "internal.hpp"

namespace bkts {

bkts_tc tc_create(bkts_ctx ctx, const bkts_tc_desc* d);

}  // namespace bkts
