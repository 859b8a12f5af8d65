"""MI355X-native cascading-bit-array minimal perfect hash function.

The compute path lives in the HIP library ``libmphf.so`` (built from
``csrc/``); :mod:`paper_1702_03154_amd.mphf` is the thin ctypes binding over its
C ABI.  Importing this package loads nothing: the binding loads the library on
first use and raises if it is missing.
"""
