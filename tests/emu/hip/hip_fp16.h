#pragma once
#include <cstring>
struct __half { unsigned short u; };
inline float __half2float(__half h) { _Float16 f; std::memcpy(&f, &h.u, 2); return (float)f; }
inline __half __float2half_rn(float v) { _Float16 f = (_Float16)v; __half h; std::memcpy(&h.u, &f, 2); return h; }
inline __half __ushort_as_half(unsigned short u) { return __half{u}; }
inline unsigned short __half_as_ushort(__half h) { return h.u; }
