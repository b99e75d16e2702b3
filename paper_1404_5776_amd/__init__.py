"""MI355X-native truncated block-sparse density-matrix RT-TDDFT propagation."""
