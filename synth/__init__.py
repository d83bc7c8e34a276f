"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This package holds *no* arithmetic of the hash method.  It only draws
numbers:

* ``synth.constants`` draws the instance parameters of Poseidon-12 that the
  paper never prints (its Alg. 1 names the round constants ``C`` and the
  matrix ``M`` but gives no values): 30 x 12 round constants uniform in
  [0, p) and the first row of a 12 x 12 circulant with entries in [1, 64].
  They are stored once in ``poseidon12.json``; both sides read that file.
* ``synth.inputs`` is a counter-based generator of uniform Goldilocks words
  (SplitMix64 finaliser of Steele, Lea and Flood, 2014) and of the shape
  streams of the batched and served workloads.

The only comparison with p here is rejection sampling (keep a draw if it is
below p), which is sampling, not field arithmetic.
"""

from .inputs import (  # noqa: F401
    GOLDILOCKS_P,
    goldilocks_words,
    leaves_colmajor,
    splitmix64_mix,
)
