// Test shim: the plain launch's tile schedule (ktau_order.h) on the host.
#include "ktau_order.h"

extern "C" void order_tile(long long w, long long T, long long b, long long* yq, long long* xq) {
  int64_t y, x;
  ktau::scheduled_tile(w, T, b, y, x);
  *yq = y;
  *xq = x;
}
