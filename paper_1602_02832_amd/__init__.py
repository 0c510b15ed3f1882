"""Tree/Hermite block-step force evaluation on MI355X (gfx950).

Modules:
  workloads  seeded synthetic inputs (Plummer, Salpeter, configurations)
  binding    ctypes binding over libhtree.so / libhtree_host.so
  driver     tree/Hermite integrator with the force on the GPU
  build      compiles the native libraries in-tree

Nothing is loaded at import time; the binding loads the native libraries on
first use and raises if they are not built.
"""
