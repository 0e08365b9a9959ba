// CPU model of the cooperative sweep's per-move agreement protocol (spread
// walkers): C workers, one per slice, each publishes its partial sum of a
// micro-update to a mailbox slot chosen by the parity of the move counter,
// releases it with one fetch-add on an arrival counter, waits (bounded: at most
// cap polls) until the counter reaches C * (moves so far), then adds the C
// partials in slice order.  The model checks that every worker sees every
// move's total, bitwise the same and equal to the sum in slice order, and
// that a worker that stops arriving makes the others give up (status set),
// with every worker leaving.
//
//   spread_protocol_model C MOVES CAP STALL_AT
//     STALL_AT < 0: no stall; else worker C-1 stops before move STALL_AT.
// Prints "ok <moves agreed>" or "gaveup <moves agreed by all> <workers left>".
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

int main(int argc, char **argv)
{
    const int C = atoi(argv[1]), moves = atoi(argv[2]);
    const unsigned cap = (unsigned)atol(argv[3]);
    const int stall_at = atoi(argv[4]);
    std::vector<std::atomic<double>> mail(2 * C);
    std::atomic<unsigned> arrive{0}, status{0}, left{0};
    std::vector<std::vector<double>> seen(C, std::vector<double>(moves, 0.0));
    std::vector<int> done(C, 0);
    auto partial = [](int g, int mv) { return 1.0 / (1.0 + g) + 1e-3 * mv * (g + 1); };
    auto worker = [&](int g) {
        for (int mv = 0; mv < moves; ++mv) {
            if (g == C - 1 && stall_at >= 0 && mv == stall_at)
                break;   // this worker stops arriving
            mail[(mv & 1) * C + g].store(partial(g, mv), std::memory_order_relaxed);
            arrive.fetch_add(1, std::memory_order_release);
            const unsigned target = (unsigned)(mv + 1) * (unsigned)C;
            unsigned spins = 0;
            bool gave_up = false;
            while (arrive.load(std::memory_order_acquire) < target) {
                if (++spins > cap) {
                    gave_up = true;
                    break;
                }
                std::this_thread::yield();
            }
            if (gave_up) {
                status.fetch_or(1);
                break;
            }
            double tot = 0.0;
            for (int q = 0; q < C; ++q)
                tot += mail[(mv & 1) * C + q].load(std::memory_order_relaxed);
            seen[g][mv] = tot;
            done[g] = mv + 1;
        }
        left.fetch_add(1);
    };
    std::vector<std::thread> th;
    for (int g = 0; g < C; ++g)
        th.emplace_back(worker, g);
    for (auto &t : th)
        t.join();
    int agreed = moves;
    for (int g = 0; g < C; ++g)
        agreed = done[g] < agreed ? done[g] : agreed;
    for (int mv = 0; mv < agreed; ++mv) {
        double want = 0.0;
        for (int q = 0; q < C; ++q)
            want += partial(q, mv);
        for (int g = 0; g < C; ++g)
            if (seen[g][mv] != want) {
                printf("mismatch move %d worker %d\n", mv, g);
                return 1;
            }
    }
    if (status.load())
        printf("gaveup %d %u\n", agreed, left.load());
    else
        printf("ok %d\n", agreed);
    return 0;
}
