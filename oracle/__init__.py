"""CPU oracle -- TEST INFRASTRUCTURE, not part of the product.

Plain, slow, obviously correct CPU implementations of what the compressed
stage loop computes, used only by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``.  Nothing in the product package imports
this package, and this package imports nothing from the product package.

* :mod:`oracle.sim`      -- FP64 numpy simulator, gate matrices, closed forms
                            (GHZ, QFT of basis/product states, QAOA ring
                            transfer matrix), dense Kronecker brute force,
                            fidelity.
* :mod:`oracle.planner`  -- Algorithm 1 circuit partition, inner/outer sets
                            and SV groups (paper Section 4.1).
* :mod:`oracle.native`   -- ctypes loader for the C parts: ``codec_ref.c``
                            (point-wise error-bounded codec, Section 4.3,
                            Algorithm 2) and ``sim_ref.c`` (OpenMP FP64
                            simulator and the QFT closed form).
"""
