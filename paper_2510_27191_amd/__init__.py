"""MI355X-native hot path of Vectorized Online POMDP Planning (VOPP).

The planner itself lives in the HIP library ``libvopp.so`` (built from
``csrc/``) behind the C ABI declared in ``include/vopp.h``; ``vopp`` is the
thin ctypes binding.  ``instances`` generates seeded synthetic POMDPs.
Importing this package loads nothing.
"""
