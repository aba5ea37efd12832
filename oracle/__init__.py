"""CPU FP64 oracle for the time-stepping resolvent method (Martini, Rodriguez, Towne & Cavalieri,
"Efficient computation of global resolvent modes").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or execute this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.
It shares no code, tables or helpers with the HIP library; the two meet only through the seeded
inputs of ``workloads.py`` (which holds none of the method's arithmetic).

Everything here is plain NumPy / SciPy in float64 / complex128, written to be checked against the
paper by eye rather than to be fast:

* ``operators``  -- the linear operators L (the paper's -A) as sparse matrices, built straight from
                    their PDE definitions with second-order central differences.
* ``dense``      -- the textbook ground truth: the resolvent (i w I - L)^{-1} and its SVD (Sec. 2.1),
                    and the exact transfer matrix of the RK4-discretised system (its fully discrete limit).
* ``stepping``   -- explicit RK4 time marching of the direct and adjoint systems with all frequencies
                    forced at once and projected by a Fourier sum: the transient-response method with a
                    one-window forcing (Sec. 2.2) and the steady-state-response method (Sec. 2.3).
* ``iteration``  -- the block power iteration with frequency-domain normalisation and the Rayleigh-Ritz
                    gain/mode estimates of Appendix A.
* ``gradient``   -- gain sensitivity to the reaction field mu: the closed form from the SVD and
                    finite differences of the discrete gain.
* ``krylov``     -- block Arnoldi estimates on the steady-state response (Appendix A).
* ``weights``    -- diagonal input and output matrices B, C and metrics W_f, W_y (Sec. 2.1).
* ``trm``        -- the transient-response method with time-domain hand-off: runs forced by sampled signals
                    interpolated between samples (App. C), FIR flattening filters (App. B) and the power
                    iteration that hands the adjoint output back in time (Sec. 2.2).

Parity pins for every function are in ``tests/test_oracle_*.py``.  Functions without such a pin say
"parity unpinned" in their docstring (there are none at present).
"""
