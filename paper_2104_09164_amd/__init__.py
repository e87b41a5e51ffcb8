"""MI355X-native encrypted dense-network inference over RNS-CKKS.

Hot path (homomorphic evaluation of dense layers with x^2 activations on
slot-packed ciphertexts) runs in hand-written HIP kernels for gfx950 inside
``libhe.so`` behind the C ABI of ``include/he.h``:

  he        ctypes binding of the C ABI (torch supplies device memory/streams)
  synth     seeded synthetic workloads (weights, inputs, uniform residues)
  netplan   host-side network plan: levels, scales, rotation steps per layer
  batch     batched evaluation of whole networks and graph replay
  serve     continuous-batching request loop with HBM-footprint admission
  tune      autotuner of bit-preserving launch choices

Importing this package loads nothing; ``he.lib()`` loads the library and
raises if it is not built.
"""
