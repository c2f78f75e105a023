"""Replica-averaged Brownian dynamics on MI355X (gfx950).

The GPU library lives in ``csrc/`` behind the C ABI declared in
``include/ra.h``; ``ra`` is its thin Python binding. ``workloads`` holds the
seeded synthetic inputs. Nothing is loaded at import time.
"""
