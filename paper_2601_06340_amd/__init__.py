"""MI355X-native two-beam FFT beam propagation (dynamical X-ray diffraction).

The hot path (plan setup, batched FFT march, coupling, reflectivity) runs in the
HIP library ``libbpm_hip.so`` built from ``csrc/``; ``bpm`` is its ctypes
binding, ``synth`` builds seeded synthetic inputs.  Nothing is imported eagerly.
"""
__all__ = ["bpm", "synth"]
