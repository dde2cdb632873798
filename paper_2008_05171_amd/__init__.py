"""MI355X-native FastPAM1 / eager FastPAM2 k-medoids (package stub)."""
