"""Reference oracle for the forward-folding likelihood: TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 CPU implementation of one model evaluation of the
forward-folding profile-likelihood fit (paper: "General concept and statistical
methods", Eq. 3-9, and "Structure of the framework", the three-step signal
calculation), written from the paper for checking the HIP engine. Only the
tests, the package's smoke check and the benchmark's CPU-baseline leg may
import it; the engine never does, and the two share no code.

Every function cites the passage it follows. Readings of points the paper
leaves open are listed in the design notes and repeated where they are used.

Modules
  oscillation  survival probabilities (Eq. 1, exact three-flavour, Eq. 10)
  model        parsing of the model description (parameters, datasets)
  fold         event binning and the per-event oscillation weighting (step 1)
  spectrum     rescale (step 2), energy-scale re-binning (step 3), backgrounds
  likelihood   Poisson deviance, priors, full evaluation, complex-step gradient
  fit          minimisation, EDM, profile scans
"""
