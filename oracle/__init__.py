"""Plain FP64 CPU oracle of the DeepABM-COVID daily transmission-and-progression step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import anything from here.  The oracle shares no code
with the GPU library (no kernels, headers, tables or helpers); both receive the same
seeded inputs from ``synthpop``.

Modules (each function cites the passage of the paper it follows):

* ``philox``  -- Philox-NxW counter-based generator (Salmon et al., SC'11) and the
  uniform / Poisson / partner mappings of the random-number layout.
* ``tables``  -- the Gamma infectiousness integral of eq. 1, per-stage factors,
  Poisson thresholds.
* ``graph``   -- the daily contact graph (section 3, "Interaction Networks").
* ``step``    -- eq. 1-2 transmission, disease progression (section 3) and the
  interventions of section 4 and the case study of section 5.
* ``soft``    -- the relaxed (Gumbel-softmax) forward step with forward-mode
  tangents for the gradient with respect to R and the age susceptibilities.
* ``mlp``     -- FP64 reference of the calibration network.

Functions whose result has no independent pin say "parity unpinned" in their
docstring.
"""
