// q2x_build_id.cpp -- the library's build identity (a hash of its sources,
// defined by the build script), part of the batch tuning cache key.
#ifndef Q2X_BUILD_ID
#error "Q2X_BUILD_ID is defined by the build script"
#endif

extern "C" const char* q2x_build_id(void) { return Q2X_BUILD_ID; }
