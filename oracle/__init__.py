"""CPU FP64 oracle of the HSDE-ADMM for chordally sparse SDPs.

TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import, call or execute anything in this package; the
GPU library never does, and this package never imports the GPU library.
"""
