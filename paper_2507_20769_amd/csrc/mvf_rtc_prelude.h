// mvf_rtc_prelude.h -- the few C library names the device headers use, for
// compilation with hiprtc (which provides no C headers; its fixed-width types
// live in a namespace).  Included only when __HIPCC_RTC__ is defined.
#pragma once
typedef __hip_internal::int8_t int8_t;
typedef __hip_internal::uint8_t uint8_t;
typedef __hip_internal::int16_t int16_t;
typedef __hip_internal::uint16_t uint16_t;
typedef __hip_internal::int32_t int32_t;
typedef __hip_internal::uint32_t uint32_t;
typedef __hip_internal::int64_t int64_t;
typedef __hip_internal::uint64_t uint64_t;
typedef struct ihipStream_t *hipStream_t;
typedef struct ihipEvent_t *hipEvent_t;
#ifndef INT64_MAX
#define INT64_MAX 0x7fffffffffffffffLL
#endif
