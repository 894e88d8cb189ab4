"""FRUITNINJA edge timing and validation on MI355X (gfx950).

The HIP library and its ctypes binding live in ``fn``; ``workload`` holds
the seeded synthetic inputs.  Importing the package loads nothing native:
``fn`` loads ``libfruitninja.so`` on first use and raises if it is missing.
"""
