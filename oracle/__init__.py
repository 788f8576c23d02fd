"""CPU oracle for the CT-AUX walker (Hahner et al., DCA++, Sec. 2.3).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP library under
``paper_1901_01047_amd/`` and never imports it.

Everything here is plain NumPy in float64 and deliberately slow:

* ``geometry``  -- periodic cluster sites and momenta from superlattice vectors.
* ``g0``        -- bare cluster propagator of the isolated periodic cluster.
* ``ed``        -- exact diagonalisation of small Hubbard clusters (test oracle).
* ``fock``      -- brute-force Fock-space trace of a time-ordered product.
* ``ctaux``     -- the single-vertex CT-AUX Markov chain (insert / remove,
                   bordered-inverse and cofactor updates, direct re-inversion).
* ``measure``   -- direct non-uniform Fourier measurement of M and the
                   Green's function estimator G = G0 - G0 <M> G0 / beta.
* ``stats``     -- binning and jackknife error bars.

Pins that fix each function independently of itself live in
``tests/test_oracle_*.py``.  One result is "parity unpinned": G(K, i w_n) for
the 4x4 and larger clusters, where no exact diagonalisation is feasible; it is
pinned only indirectly (direct-inversion invariant, K-independence, agreement
of the same estimator with ED on the 2x2 cluster).
"""
