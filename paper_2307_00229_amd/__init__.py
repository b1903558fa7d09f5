"""MI355X-native C-l-AIR restriction setup (constrained local approximate ideal restriction).

The package holds the HIP library (``csrc/``, built into ``libclair.so``), its
thin ctypes binding (``clair``) and the seeded synthetic input generators
(``problems``).
"""
