"""CPU oracle for encrypted dense-network inference over RNS-CKKS.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import, call, link or execute anything in
this package.  The GPU library under ``paper_2104_09164_amd/`` never does, and
the two share no code: this package computes every expected value from the
paper's definitions in plain C++ (``cpp/ckks_oracle.cpp``, unsigned 128-bit
products reduced with ``%``) and plain numpy FP64 (encoder, decoder, plaintext
network), plus an independent pure-Python big-integer twin (``tiny.py``) for
ring dimensions up to 64.

Modules:
  params    prime chains and parameter presets (deterministic Miller-Rabin)
  encode    CKKS canonical-embedding encoder/decoder (FFT and direct forms)
  plan      dense-layer plan: diagonals, baby/giant pre-rotation, rotation steps
  plainnet  FP64 plaintext network (the accuracy reference)
  ckks      ctypes driver of the C++ core: keygen, encrypt, decrypt, all ops
  tiny      independent big-integer oracle for N <= 64
"""
