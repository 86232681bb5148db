"""MI355X-native SDC-resilient error-bounded lossy compressor (arXiv 2010.03144).

Modules:
  sdcsz  -- Python binding of the C ABI (include/sdcsz.h) over libsdcsz.so
  synth  -- seeded synthetic fields and fault plans
  build  -- hipcc build of the library for gfx950
"""
