// No-op roctx ranges for the host-only scheduler build.
#pragma once
inline int roctxRangePushA(const char*) { return 0; }
inline int roctxRangePop() { return 0; }
