// Force-included into the ThreadSanitizer build of the scheduler test.
// libstdc++ 11 waits on a condition variable with pthread_cond_clockwait,
// which this toolchain's ThreadSanitizer runtime does not intercept: it then
// misses that the wait releases the mutex, and reports every later use of
// that mutex as a double lock or a race.  Without the macro, libstdc++
// waits through pthread_cond_timedwait, which it does intercept.
#pragma once
#include <bits/c++config.h>
#undef _GLIBCXX_USE_PTHREAD_COND_CLOCKWAIT
