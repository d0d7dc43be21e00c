"""MI355X-native QTT fractional-step library (arxiv 2507.05222): HIP kernels in
libqtt.so behind a C ABI (include/qtt.h), with a thin ctypes binding in qtt.py."""
