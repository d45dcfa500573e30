"""libsrw: exact shortest reset words (bidirectional subset BFS) on MI355X.

Submodules:
  srw     ctypes binding of the C ABI (include/srw.h); loads libsrw.so
  inputs  seeded synthetic automata (random uniform, Černý)
  build   compiles libsrw.so for gfx950 with hipcc
"""
