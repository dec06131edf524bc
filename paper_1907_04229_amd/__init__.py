"""MI355X-native CPTR-FGMRES: two-stage constrained pressure-temperature residual
preconditioning of fully implicit thermal multiphase Jacobians on gfx950."""
